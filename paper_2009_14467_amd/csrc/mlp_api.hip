// C ABI of the learned pre-alignment filter, and its use inside a search.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "mlp.hpp"
#include "prim.hpp"

namespace pastis {
namespace {

constexpr int kMaxBatch = 65536;

pastis_status mlp_alloc(pastis_ctx *ctx) {
    if (ctx->mlp_alloc) return PASTIS_OK;
    MlpState &S = ctx->mlp;
    auto grab = [&](void **p, size_t bytes) -> pastis_status {
        if (*p) return PASTIS_OK;  // kept from an earlier, partly failed call
        if (hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return set_error(ctx, PASTIS_E_NOMEM, "network allocation failed");
        }
        return PASTIS_OK;
    };
    PASTIS_TRY(grab((void **)&S.theta, sizeof(float) * kMlpParams));
    PASTIS_TRY(grab((void **)&S.m, sizeof(float) * kMlpParams));
    PASTIS_TRY(grab((void **)&S.v, sizeof(float) * kMlpParams));
    PASTIS_TRY(grab((void **)&S.grad, sizeof(float) * kMlpParams));
    PASTIS_TRY(grab((void **)&S.W1b, 2 * kMlpHidden * kMlpIn));
    PASTIS_TRY(grab((void **)&S.W2b, 2 * kMlpHidden * kMlpHidden));
    PASTIS_TRY(grab((void **)&S.W2Tb, 2 * kMlpHidden * kMlpHidden));
    PASTIS_TRY(grab((void **)&S.w3b, 2 * kMlpHidden));
    PASTIS_TRY(grab((void **)&S.mean, sizeof(float) * kMlpIn));
    PASTIS_TRY(grab((void **)&S.stdv, sizeof(float) * kMlpIn));
    PASTIS_TRY(grab((void **)&S.moments, sizeof(double) * 2 * kMlpIn));
    S.batch_cap = kMaxBatch;
    PASTIS_TRY(grab((void **)&S.ZT, 2 * (size_t)kMlpIn * kMaxBatch));
    PASTIS_TRY(grab((void **)&S.H1, 2 * (size_t)kMlpHidden * kMaxBatch));
    PASTIS_TRY(grab((void **)&S.DH2, 2 * (size_t)kMlpHidden * kMaxBatch));
    PASTIS_TRY(grab((void **)&S.DH1, 2 * (size_t)kMlpHidden * kMaxBatch));
    PASTIS_TRY(grab((void **)&S.part, sizeof(float) * (size_t)(kMaxBatch / (16 * kMlpTrainWaves)) * kMlpPartN));
    PASTIS_TRY(grab((void **)&S.wpart, sizeof(float) * (size_t)(kMaxBatch / kMlpSplitK) *
                                           (kMlpHidden * kMlpHidden + kMlpHidden * kMlpIn)));
    ctx->mlp_alloc = true;
    return PASTIS_OK;
}

pastis_status need_net(pastis_ctx *ctx) {
    if (!ctx->mlp_set) return set_error(ctx, PASTIS_E_STATE, "no network: call pastis_mlp_set first");
    return PASTIS_OK;
}

}  // namespace

void mlp_free(pastis_ctx *ctx) {
    MlpState &S = ctx->mlp;
    void *ps[] = {S.theta, S.m, S.v, S.grad, S.W1b, S.W2b, S.W2Tb, S.w3b, S.mean, S.stdv, S.moments,
                  S.ZT, S.H1, S.DH2, S.DH1, S.part, S.wpart, S.pool_X, S.pool_y};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    S = MlpState{};
    ctx->mlp_alloc = false;
}

// Filter the ctx's candidates in place (stable); returns the kept count.
pastis_status mlp_filter_candidates(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n,
                                   hipStream_t s) {
    PASTIS_TRY(need_net(ctx));
    const int64_t nc = ctx->n_candidates;
    if (nc == 0) return PASTIS_OK;
    HIP_TRY(ctx, stage_begin(ctx, kStLearned, s), "event");
    void *comp, *feat, *logit, *keep, *pos, *tmp, *temp;
    PASTIS_TRY(ensure(ctx, kBufMlpComp, sizeof(float) * 10 * (size_t)std::max<int64_t>(n, 1), &comp));
    PASTIS_TRY(ensure(ctx, kBufMlpFeat, sizeof(float) * kMlpIn * (size_t)nc, &feat));
    PASTIS_TRY(ensure(ctx, kBufMlpLogit, sizeof(float) * (size_t)nc, &logit));
    PASTIS_TRY(ensure(ctx, kBufMlpKeep, (size_t)nc + 8, &keep));
    PASTIS_TRY(ensure(ctx, kBufMlpPos, sizeof(uint32_t) * ((size_t)nc + 1), &pos));
    PASTIS_TRY(ensure(ctx, kBufMlpTmp, sizeof(uint32_t) * 5 * (size_t)nc, &tmp));
    PASTIS_TRY(ensure(ctx, kBufMlpOrder, scan_temp_bytes(nc) + 256, &temp));
    const uint32_t *cand[5] = {(const uint32_t *)ctx->buf[kBufCandLo].ptr, (const uint32_t *)ctx->buf[kBufCandHi].ptr,
                               (const uint32_t *)ctx->buf[kBufCandCnt].ptr, (const uint32_t *)ctx->buf[kBufCandS1].ptr,
                               (const uint32_t *)ctx->buf[kBufCandS2].ptr};
    HIP_TRY(ctx,
            mlp_features(codes, st.d_off, n, cand[0], cand[1], cand[2], cand[3], cand[4], nc, (float *)comp,
                         (float *)feat, s),
            "feature kernels");
    HIP_TRY(ctx, mlp_forward(ctx->mlp, (const float *)feat, nc, (float *)logit, s), "network kernel");
    HIP_TRY(ctx, mlp_keep((const float *)logit, nc, ctx->mlp_tau, (uint8_t *)keep, s), "keep kernel");
    uint32_t *p32 = (uint32_t *)pos;
    HIP_TRY(ctx, (exclusive_scan<uint8_t, uint32_t>((const uint8_t *)keep, nc, p32, p32 + nc, temp, s)), "scan");
    uint32_t *t32 = (uint32_t *)tmp;
    uint32_t *outs[5] = {t32, t32 + nc, t32 + 2 * nc, t32 + 3 * nc, t32 + 4 * nc};
    HIP_TRY(ctx, compact5((const uint8_t *)keep, p32, nc, cand, outs, s), "compact kernel");
    uint32_t kept = 0;
    PASTIS_TRY(read_device(ctx, p32 + nc, &kept, sizeof(kept), s));
    for (int f = 0; f < 5; ++f)
        if (kept)
            HIP_TRY(ctx, hipMemcpyAsync((void *)cand[f], outs[f], sizeof(uint32_t) * kept, hipMemcpyDeviceToDevice, s),
                    "copy");
    HIP_TRY(ctx, stage_end(ctx, kStLearned, s), "event");
    ctx->n_candidates = kept;
    return PASTIS_OK;
}

pastis_status set_network(pastis_ctx *ctx, const float *params, const float *mean, const float *stdv, float tau);
pastis_status run_epoch(pastis_ctx *ctx, const float *X, const uint8_t *labels, const int32_t *order, int64_t n,
                        int32_t batch, float lr, float pos_weight, float *mean_loss, hipStream_t s);
pastis_status calibrate_tau(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n, double target,
                            float *tau, hipStream_t s);

}  // namespace pastis

using namespace pastis;

extern "C" {

pastis_status pastis_mlp_set(pastis_ctx *ctx, const float *params, const float *mean, const float *stdv, float tau) {
    if (!ctx || !params || !mean || !stdv) return PASTIS_E_INVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return set_network(ctx, params, mean, stdv, tau);
}

}  // extern "C"

namespace pastis {

pastis_status set_network(pastis_ctx *ctx, const float *params, const float *mean, const float *stdv, float tau) {
    PASTIS_TRY(mlp_alloc(ctx));
    MlpState &S = ctx->mlp;
    for (int f = 0; f < kMlpIn; ++f)
        if (!(stdv[f] > 0.f)) return set_error(ctx, PASTIS_E_INVAL, "std must be positive");
    HIP_TRY(ctx, hipMemcpy(S.theta, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice), "copy");
    HIP_TRY(ctx, hipMemcpy(S.mean, mean, sizeof(float) * kMlpIn, hipMemcpyHostToDevice), "copy");
    HIP_TRY(ctx, hipMemcpy(S.stdv, stdv, sizeof(float) * kMlpIn, hipMemcpyHostToDevice), "copy");
    HIP_TRY(ctx, fill<uint32_t>((uint32_t *)S.m, kMlpParams, 0u, nullptr), "reset");
    HIP_TRY(ctx, fill<uint32_t>((uint32_t *)S.v, kMlpParams, 0u, nullptr), "reset");
    HIP_TRY(ctx, mlp_refresh(S, nullptr), "refresh");
    HIP_TRY(ctx, hipDeviceSynchronize(), "sync");
    ctx->mlp_tau = tau;
    ctx->mlp_step = 0;
    ctx->mlp_set = true;
    return PASTIS_OK;
}

// Minibatch gradient + Adam over order[0..n) (indices already checked).
pastis_status run_epoch(pastis_ctx *ctx, const float *X, const uint8_t *labels, const int32_t *order, int64_t n,
                        int32_t batch, float lr, float pos_weight, float *mean_loss, hipStream_t s) {
    const int64_t nb = (n + batch - 1) / batch;
    void *lossd = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpLogit, sizeof(float) * (size_t)(nb + 1), &lossd));
    HIP_TRY(ctx, fill<uint32_t>((uint32_t *)lossd, nb, 0u, s), "reset");
    HIP_TRY(ctx, mlp_refresh(ctx->mlp, s), "refresh");
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t off = b * batch, cnt = std::min<int64_t>(batch, n - off);
        const int B = (int)((cnt + 15) / 16 * 16);
        HIP_TRY(ctx,
                mlp_batch_grad(ctx->mlp, X, labels, order, off, cnt, B, pos_weight, (float *)lossd + b, lr,
                               ++ctx->mlp_step, s),
                "gradient and Adam kernels");
    }
    std::vector<float> h((size_t)nb);
    PASTIS_TRY(read_device(ctx, lossd, h.data(), sizeof(float) * nb, s));
    double acc = 0.0;
    for (float v : h) acc += v;
    if (mean_loss) *mean_loss = (float)(acc / (double)nb);
    return PASTIS_OK;
}

// Logits of X [n] into the logit buffer, copied to the host with the labels.
pastis_status logits_to_host(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n,
                             std::vector<float> &y, std::vector<uint8_t> &t, hipStream_t s) {
    void *logit = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpLogit, sizeof(float) * (size_t)n, &logit));
    HIP_TRY(ctx, mlp_forward(ctx->mlp, X, n, (float *)logit, s), "network kernel");
    y.resize((size_t)n);
    t.resize((size_t)n);
    PASTIS_TRY(read_device(ctx, logit, y.data(), sizeof(float) * n, s));
    PASTIS_TRY(read_device(ctx, labels, t.data(), (size_t)n, s));
    return PASTIS_OK;
}

// The logit threshold keeping at least target of the positives of X / labels.
pastis_status calibrate_tau(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n, double target,
                            float *tau, hipStream_t s) {
    std::vector<float> y;
    std::vector<uint8_t> t;
    PASTIS_TRY(logits_to_host(ctx, X, labels, n, y, t, s));
    std::vector<float> pos;
    for (int64_t q = 0; q < n; ++q)
        if (t[q]) pos.push_back(y[q]);
    if (pos.empty()) return set_error(ctx, PASTIS_E_INVAL, "no positive examples");
    std::sort(pos.begin(), pos.end());
    // keep logit >= tau for at least target of the positives
    const size_t miss = (size_t)((1.0 - target) * (double)pos.size());
    *tau = pos[std::min(miss, pos.size() - 1)];
    ctx->mlp_tau = *tau;
    return PASTIS_OK;
}

}  // namespace pastis

extern "C" {

pastis_status pastis_mlp_get(pastis_ctx *ctx, float *params, float *mean, float *stdv, float *tau) {
    if (!ctx) return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(ctx, hipDeviceSynchronize(), "sync");
    MlpState &S = ctx->mlp;
    if (params) HIP_TRY(ctx, hipMemcpy(params, S.theta, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "copy");
    if (mean) HIP_TRY(ctx, hipMemcpy(mean, S.mean, sizeof(float) * kMlpIn, hipMemcpyDeviceToHost), "copy");
    if (stdv) HIP_TRY(ctx, hipMemcpy(stdv, S.stdv, sizeof(float) * kMlpIn, hipMemcpyDeviceToHost), "copy");
    if (tau) *tau = ctx->mlp_tau;
    return PASTIS_OK;
}

pastis_status pastis_mlp_features(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                  int input_on_device, float *features, int64_t cap, void *stream) {
    if (!ctx) return PASTIS_E_INVAL;
    if (!ctx->have_candidates) return set_error(ctx, PASTIS_E_STATE, "no candidates: call pastis_discover first");
    if (cap < ctx->n_candidates) return set_error(ctx, PASTIS_E_CAPACITY, "feature buffer too small");
    if (n != ctx->n_seqs_last) return set_error(ctx, PASTIS_E_INVAL, "sequence set differs from the discovery's");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    Staged st;
    PASTIS_TRY(stage_sequences(ctx, residues, offsets, n, input_on_device, s, st));
    unsigned long long *d_flags = nullptr, h_flags[4];
    PASTIS_TRY(reset_flags(ctx, &d_flags, s));
    uint8_t *codes = nullptr;
    PASTIS_TRY(encode_into(ctx, st.d_res, st.n_res, &codes, d_flags, s));
    PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 1, s));
    if (h_flags[0] != ~0ull) return set_error(ctx, PASTIS_E_BAD_RESIDUE, "bad residue");
    void *comp = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpComp, sizeof(float) * 10 * (size_t)std::max<int64_t>(n, 1), &comp));
    HIP_TRY(ctx,
            mlp_features(codes, st.d_off, n, (const uint32_t *)ctx->buf[kBufCandLo].ptr,
                         (const uint32_t *)ctx->buf[kBufCandHi].ptr, (const uint32_t *)ctx->buf[kBufCandCnt].ptr,
                         (const uint32_t *)ctx->buf[kBufCandS1].ptr, (const uint32_t *)ctx->buf[kBufCandS2].ptr,
                         ctx->n_candidates, (float *)comp, features, s),
            "feature kernels");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

pastis_status pastis_mlp_fit_normalizer(pastis_ctx *ctx, const float *X, int64_t n, void *stream) {
    if (!ctx || n <= 0 || !X) return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(ctx, mlp_moments(X, n, ctx->mlp.moments, ctx->mlp.mean, ctx->mlp.stdv, s), "moment kernels");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

pastis_status pastis_mlp_forward(pastis_ctx *ctx, const float *X, int64_t n, float *logits, void *stream) {
    if (!ctx || n < 0 || (n > 0 && (!X || !logits))) return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(ctx, mlp_forward(ctx->mlp, X, n, logits, s), "network kernel");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

pastis_status pastis_mlp_grad(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n, float pos_weight,
                              float *grad, float *loss, void *stream) {
    if (!ctx || n <= 0 || n > kMaxBatch || !X || !labels || !grad || !loss) return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    void *order = nullptr, *lossd = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpOrder, sizeof(int32_t) * (size_t)n, &order));
    PASTIS_TRY(ensure(ctx, kBufMlpLogit, sizeof(float) * 4, &lossd));
    HIP_TRY(ctx, iota((uint32_t *)order, n, s), "iota");
    HIP_TRY(ctx, fill<uint32_t>((uint32_t *)lossd, 1, 0u, s), "reset");
    const int B = (int)((n + 15) / 16 * 16);
    HIP_TRY(ctx, mlp_refresh(ctx->mlp, s), "refresh");
    HIP_TRY(ctx,
            mlp_batch_grad(ctx->mlp, X, labels, (const int32_t *)order, 0, n, B, pos_weight, (float *)lossd, 0.f, 0, s),
            "gradient kernels");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    HIP_TRY(ctx, hipMemcpy(grad, ctx->mlp.grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "copy");
    HIP_TRY(ctx, hipMemcpy(loss, lossd, sizeof(float), hipMemcpyDeviceToHost), "copy");
    return PASTIS_OK;
}

pastis_status pastis_mlp_train_epoch(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n_examples,
                                     const int32_t *order, int64_t n, int32_t batch, float lr, float pos_weight,
                                     float *mean_loss, void *stream) {
    if (!ctx || n <= 0 || n_examples <= 0 || !X || !labels || !order || batch < 16 || batch % 16 ||
        batch > kMaxBatch)
        return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    {
        unsigned long long *d_flags = nullptr, h_flags[4];
        PASTIS_TRY(reset_flags(ctx, &d_flags, s));
        HIP_TRY(ctx, mlp_check_order(order, n, n_examples, d_flags, s), "index check kernel");
        PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 1, s));
        if (h_flags[0] != ~0ull) return set_error(ctx, PASTIS_E_INVAL, "order holds an index outside [0, n_examples)");
    }
    return run_epoch(ctx, X, labels, order, n, batch, lr, pos_weight, mean_loss, s);
}

pastis_status pastis_mlp_calibrate(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n,
                                   double target_recall, float *tau, void *stream) {
    if (!ctx || n <= 0 || !X || !labels || !tau || !(target_recall > 0.0 && target_recall <= 1.0))
        return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return calibrate_tau(ctx, X, labels, n, target_recall, tau, s);
}

}  // extern "C"

// ---------------------------------------------------------------- training in the library

namespace pastis {
namespace {

// splitmix64 (Steele, Lea and Flood, 2014): the shuffle keys and initial weights
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// keys[q] = random 32 bits of (seed, round, vals[q]); the sort by them is a
// seeded permutation of vals
__global__ void shuffle_keys_kernel(const int32_t *__restrict__ vals_in, int64_t n, uint64_t seed, uint64_t round,
                                    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = vals_in ? (uint32_t)vals_in[q] : (uint32_t)q;
        keys[q] = mix64(seed ^ mix64(round * 0x100000001B3ull + v)) >> 32;
        vals[q] = v;
    }
}

__global__ void gather_kernel(const float *__restrict__ X, const uint8_t *__restrict__ y,
                              const uint32_t *__restrict__ idx, int64_t n, float *__restrict__ Xo,
                              uint8_t *__restrict__ yo) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n * kMlpIn;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / kMlpIn;
        const int f = (int)(q % kMlpIn);
        const uint32_t src = idx[r];
        Xo[q] = X[(int64_t)src * kMlpIn + f];
        if (f == 0) yo[r] = y[src];
    }
}

__global__ void count_pos_kernel(const uint8_t *__restrict__ y, const uint32_t *__restrict__ idx, int64_t n,
                                 unsigned long long *__restrict__ out) {
    unsigned long long c = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        c += y[idx[q]] != 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ void labels_kernel(const pastis_pair_record *__restrict__ rec, int64_t n, uint8_t *__restrict__ y) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        y[q] = rec[q].passed != 0;
}

inline unsigned blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

// Buffers of one training call, released on return.
struct TrainBufs {
    std::vector<void *> ptrs;
    ~TrainBufs() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    pastis_status get(pastis_ctx *ctx, int64_t count, T **out) {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ctx, PASTIS_E_NOMEM, "training buffer allocation failed");
        }
        ptrs.push_back(p);
        *out = (T *)p;
        return PASTIS_OK;
    }
};

// A seeded permutation of vals_in[0..n) (or of 0..n when vals_in is NULL) into out.
pastis_status shuffle(pastis_ctx *ctx, TrainBufs &tb, const int32_t *vals_in, int64_t n, uint64_t seed,
                      uint64_t round, uint32_t *out, hipStream_t s) {
    uint64_t *k0, *k1;
    uint32_t *v1;
    char *temp;
    PASTIS_TRY(tb.get(ctx, n, &k0));
    PASTIS_TRY(tb.get(ctx, n, &k1));
    PASTIS_TRY(tb.get(ctx, n, &v1));
    PASTIS_TRY(tb.get(ctx, (int64_t)radix_temp_bytes(n) + 256, &temp));
    shuffle_keys_kernel<<<blocks_for(n), 256, 0, s>>>(vals_in, n, seed, round, k0, out);
    HIP_TRY(ctx, hipGetLastError(), "shuffle kernel");
    bool alt = false;
    HIP_TRY(ctx, radix_sort(k0, out, k1, v1, n, 32, temp, s, &alt), "sort");
    if (alt) HIP_TRY(ctx, hipMemcpyAsync(out, v1, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s), "copy");
    return PASTIS_OK;
}

// He-normal weights (Box-Muller over splitmix64), zero biases.
void initial_params(uint64_t seed, std::vector<float> &p) {
    p.assign(kMlpParams, 0.f);
    uint64_t state = seed * 0x2545F4914F6CDD1Dull + 1;
    auto uniform = [&]() {  // (0, 1]
        state = mix64(state);
        return ((double)(state >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    };
    auto normal = [&](double sd) {
        const double u1 = uniform(), u2 = uniform();
        return (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    };
    for (int t = 0; t < kMlpHidden * kMlpIn; ++t) p[kMlpOffW1 + t] = normal(std::sqrt(2.0 / kMlpIn));
    for (int t = 0; t < kMlpHidden * kMlpHidden; ++t) p[kMlpOffW2 + t] = normal(std::sqrt(2.0 / kMlpHidden));
    for (int t = 0; t < kMlpHidden; ++t) p[kMlpOffW3 + t] = normal(std::sqrt(1.0 / kMlpHidden));
}

constexpr char kMagic[8] = {'P', 'A', 'S', 'T', 'M', 'L', 'P', '1'};

}  // namespace

// Make room for `want` examples in the pool, keeping the ones it holds.
pastis_status mlp_pool_reserve(pastis_ctx *ctx, int64_t want, hipStream_t s) {
    MlpState &S = ctx->mlp;
    if (want <= S.pool_cap) return PASTIS_OK;
    const int64_t cap = std::max<int64_t>(want + want / 4, 1 << 16);
    float *X = nullptr;
    uint8_t *y = nullptr;
    if (hipMalloc(&X, sizeof(float) * kMlpIn * (size_t)cap) != hipSuccess ||
        hipMalloc(&y, (size_t)cap) != hipSuccess) {
        (void)hipGetLastError();
        if (X) (void)hipFree(X);
        return set_error(ctx, PASTIS_E_NOMEM, "example pool allocation failed");
    }
    if (S.pool_n > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(X, S.pool_X, sizeof(float) * kMlpIn * S.pool_n, hipMemcpyDeviceToDevice, s), "copy");
        HIP_TRY(ctx, hipMemcpyAsync(y, S.pool_y, (size_t)S.pool_n, hipMemcpyDeviceToDevice, s), "copy");
    }
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    if (S.pool_X) (void)hipFree(S.pool_X);
    if (S.pool_y) (void)hipFree(S.pool_y);
    S.pool_X = X;
    S.pool_y = y;
    S.pool_cap = cap;
    return PASTIS_OK;
}

// Append the features and pass/fail labels of the ctx's current candidates
// (records rec of their exact alignment) to the pool.
pastis_status mlp_pool_append(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n,
                              const pastis_pair_record *rec, hipStream_t s, int64_t *added) {
    const int64_t nc = ctx->n_candidates;
    *added = 0;
    if (nc == 0) return PASTIS_OK;
    MlpState &S = ctx->mlp;
    PASTIS_TRY(mlp_pool_reserve(ctx, S.pool_n + nc, s));
    void *comp = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpComp, sizeof(float) * 10 * (size_t)std::max<int64_t>(n, 1), &comp));
    HIP_TRY(ctx,
            mlp_features(codes, st.d_off, n, (const uint32_t *)ctx->buf[kBufCandLo].ptr,
                         (const uint32_t *)ctx->buf[kBufCandHi].ptr, (const uint32_t *)ctx->buf[kBufCandCnt].ptr,
                         (const uint32_t *)ctx->buf[kBufCandS1].ptr, (const uint32_t *)ctx->buf[kBufCandS2].ptr, nc,
                         (float *)comp, S.pool_X + (size_t)S.pool_n * kMlpIn, s),
            "feature kernels");
    labels_kernel<<<blocks_for(nc), 256, 0, s>>>(rec, nc, S.pool_y + S.pool_n);
    HIP_TRY(ctx, hipGetLastError(), "label kernel");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    S.pool_n += nc;
    *added = nc;
    return PASTIS_OK;
}

}  // namespace pastis

extern "C" {

pastis_status pastis_mlp_clear(pastis_ctx *ctx) {
    if (!ctx) return PASTIS_E_INVAL;
    ctx->mlp.pool_n = 0;
    return PASTIS_OK;
}

pastis_status pastis_mlp_pool_size(const pastis_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return PASTIS_E_INVAL;
    *n = ctx->mlp.pool_n;
    return PASTIS_OK;
}

void pastis_mlp_default_train_opts(pastis_mlp_train_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->epochs = 4;
    o->batch = 8192;
    o->lr = 2e-3f;
    o->pos_weight = 0.f;
    o->target_recall = 0.995;
    o->heldout = 0.2;
    o->seed = 0;
}

pastis_status pastis_mlp_train(pastis_ctx *ctx, const pastis_mlp_train_opts *opts, void *stream,
                               pastis_mlp_train_report *report) {
    if (!ctx) return PASTIS_E_INVAL;
    auto t0 = std::chrono::steady_clock::now();
    pastis_mlp_train_opts o;
    pastis_mlp_default_train_opts(&o);
    if (opts) o = *opts;
    if (o.epochs < 1 || o.epochs > 1000) return set_error(ctx, PASTIS_E_INVAL, "epochs must be in 1..1000");
    if (o.batch < 16 || o.batch % 16 || o.batch > kMaxBatch)
        return set_error(ctx, PASTIS_E_INVAL, "batch must be a multiple of 16 in 16..65536");
    if (!(o.lr > 0.f)) return set_error(ctx, PASTIS_E_INVAL, "lr must be > 0");
    if (!(o.target_recall > 0.0 && o.target_recall <= 1.0))
        return set_error(ctx, PASTIS_E_INVAL, "target_recall must be in (0, 1]");
    if (!(o.heldout > 0.0 && o.heldout <= 0.9)) return set_error(ctx, PASTIS_E_INVAL, "heldout must be in (0, 0.9]");
    for (int t = 0; t < 4; ++t)
        if (o.reserved[t] != 0) return set_error(ctx, PASTIS_E_INVAL, "reserved fields must be zero");
    MlpState &S = ctx->mlp;
    const int64_t n = S.pool_n;
    if (n < 64) return set_error(ctx, PASTIS_E_STATE, "the example pool holds fewer than 64 examples");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    TrainBufs tb;
    // the split: a seeded permutation, held-out share first
    uint32_t *perm;
    PASTIS_TRY(tb.get(ctx, n, &perm));
    PASTIS_TRY(shuffle(ctx, tb, nullptr, n, o.seed, 0, perm, s));
    const int64_t n_hold = std::max<int64_t>(32, (int64_t)(o.heldout * (double)n));
    const int64_t n_train = n - n_hold;
    const uint32_t *train_idx = perm + n_hold;
    unsigned long long *d_pos;
    PASTIS_TRY(tb.get(ctx, 1, &d_pos));
    HIP_TRY(ctx, fill<unsigned long long>(d_pos, 1, 0ull, s), "reset");
    count_pos_kernel<<<blocks_for(n_train), 256, 0, s>>>(S.pool_y, train_idx, n_train, d_pos);
    HIP_TRY(ctx, hipGetLastError(), "count kernel");
    unsigned long long n_pos = 0;
    PASTIS_TRY(read_device(ctx, d_pos, &n_pos, sizeof(n_pos), s));
    if (n_pos == 0) return set_error(ctx, PASTIS_E_STATE, "the training share has no positive example");
    const float pos_weight = o.pos_weight > 0.f ? o.pos_weight : (float)((double)(n_train - (int64_t)n_pos) / n_pos);
    // a fresh network; its normalisation from the training share
    std::vector<float> p0;
    initial_params(o.seed, p0);
    std::vector<float> zero(kMlpIn, 0.f), one(kMlpIn, 1.f);
    PASTIS_TRY(set_network(ctx, p0.data(), zero.data(), one.data(), 0.f));
    float *Xt;
    uint8_t *yt;
    PASTIS_TRY(tb.get(ctx, n_train * kMlpIn, &Xt));
    PASTIS_TRY(tb.get(ctx, n_train, &yt));
    gather_kernel<<<blocks_for(n_train * kMlpIn), 256, 0, s>>>(S.pool_X, S.pool_y, train_idx, n_train, Xt, yt);
    HIP_TRY(ctx, hipGetLastError(), "gather kernel");
    HIP_TRY(ctx, mlp_moments(Xt, n_train, S.moments, S.mean, S.stdv, s), "moment kernels");
    // epochs over the training share (rows of Xt / yt), reshuffled each time
    uint32_t *order;
    PASTIS_TRY(tb.get(ctx, n_train, &order));
    pastis_mlp_train_report rep{};
    for (int ep = 0; ep < o.epochs; ++ep) {
        PASTIS_TRY(shuffle(ctx, tb, nullptr, n_train, o.seed, (uint64_t)ep + 1, order, s));
        float loss = 0.f;
        PASTIS_TRY(run_epoch(ctx, Xt, yt, (const int32_t *)order, n_train, o.batch, o.lr, pos_weight, &loss, s));
        if (ep < 32) rep.epoch_loss[ep] = loss;
    }
    // tau from one half of the held-out share, recall and kept share from the other
    const int64_t n_cal = n_hold / 2, n_test = n_hold - n_cal;
    float *Xh;
    uint8_t *yh;
    PASTIS_TRY(tb.get(ctx, n_hold * kMlpIn, &Xh));
    PASTIS_TRY(tb.get(ctx, n_hold, &yh));
    gather_kernel<<<blocks_for(n_hold * kMlpIn), 256, 0, s>>>(S.pool_X, S.pool_y, perm, n_hold, Xh, yh);
    HIP_TRY(ctx, hipGetLastError(), "gather kernel");
    float tau = 0.f;
    PASTIS_TRY(calibrate_tau(ctx, Xh, yh, n_cal, o.target_recall, &tau, s));
    std::vector<float> y;
    std::vector<uint8_t> t;
    PASTIS_TRY(logits_to_host(ctx, Xh + (size_t)n_cal * kMlpIn, yh + n_cal, n_test, y, t, s));
    int64_t pos = 0, pos_kept = 0, kept = 0;
    for (int64_t q = 0; q < n_test; ++q) {
        const bool k = y[q] >= tau;
        kept += k;
        pos += t[q] != 0;
        pos_kept += (t[q] != 0) && k;
    }
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    rep.n_examples = n;
    rep.n_train = n_train;
    rep.n_positive = (int64_t)n_pos;
    rep.pos_weight = pos_weight;
    rep.tau = tau;
    rep.heldout_recall = pos > 0 ? (double)pos_kept / (double)pos : 1.0;
    rep.heldout_kept = n_test > 0 ? (double)kept / (double)n_test : 0.0;
    rep.epochs = o.epochs;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    return PASTIS_OK;
}

pastis_status pastis_mlp_save(pastis_ctx *ctx, const char *path) {
    if (!ctx || !path) return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    std::vector<float> p(kMlpParams), mean(kMlpIn), stdv(kMlpIn);
    float tau = 0.f;
    PASTIS_TRY(pastis_mlp_get(ctx, p.data(), mean.data(), stdv.data(), &tau));
    FILE *f = fopen(path, "wb");
    if (!f) return set_error(ctx, PASTIS_E_INVAL, std::string("cannot write ") + path);
    const int32_t head[4] = {kMlpIn, kMlpHidden, kMlpParams, 0};
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(head, sizeof(head), 1, f) == 1 &&
              fwrite(p.data(), sizeof(float), kMlpParams, f) == (size_t)kMlpParams &&
              fwrite(mean.data(), sizeof(float), kMlpIn, f) == (size_t)kMlpIn &&
              fwrite(stdv.data(), sizeof(float), kMlpIn, f) == (size_t)kMlpIn && fwrite(&tau, sizeof(float), 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok) return set_error(ctx, PASTIS_E_INVAL, std::string("write failed: ") + path);
    return PASTIS_OK;
}

pastis_status pastis_mlp_load(pastis_ctx *ctx, const char *path) {
    if (!ctx || !path) return PASTIS_E_INVAL;
    FILE *f = fopen(path, "rb");
    if (!f) return set_error(ctx, PASTIS_E_INVAL, std::string("cannot read ") + path);
    char magic[8];
    int32_t head[4];
    std::vector<float> p(kMlpParams), mean(kMlpIn), stdv(kMlpIn);
    float tau = 0.f;
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(head, sizeof(head), 1, f) == 1 &&
              head[0] == kMlpIn && head[1] == kMlpHidden && head[2] == kMlpParams &&
              fread(p.data(), sizeof(float), kMlpParams, f) == (size_t)kMlpParams &&
              fread(mean.data(), sizeof(float), kMlpIn, f) == (size_t)kMlpIn &&
              fread(stdv.data(), sizeof(float), kMlpIn, f) == (size_t)kMlpIn && fread(&tau, sizeof(float), 1, f) == 1;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after tau
    fclose(f);
    if (!ok) return set_error(ctx, PASTIS_E_INVAL, std::string("not a network file of this library: ") + path);
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return set_network(ctx, p.data(), mean.data(), stdv.data(), tau);
}

}  // extern "C"
