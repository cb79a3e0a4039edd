// C ABI of the learned pre-alignment filter, and its use inside a search.
#include <algorithm>
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
                  S.ZT, S.H1, S.DH2, S.DH1};
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

}  // namespace pastis

using namespace pastis;

extern "C" {

pastis_status pastis_mlp_set(pastis_ctx *ctx, const float *params, const float *mean, const float *stdv, float tau) {
    if (!ctx || !params || !mean || !stdv) return PASTIS_E_INVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
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
    HIP_TRY(ctx, mlp_refresh(ctx->mlp, s), "refresh");  // clears accumulated gradients
    HIP_TRY(ctx, mlp_batch_grad(ctx->mlp, X, labels, (const int32_t *)order, 0, n, B, pos_weight, (float *)lossd, s),
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
    const int64_t nb = (n + batch - 1) / batch;
    void *lossd = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpLogit, sizeof(float) * (size_t)(nb + 1), &lossd));
    {
        unsigned long long *d_flags = nullptr, h_flags[4];
        PASTIS_TRY(reset_flags(ctx, &d_flags, s));
        HIP_TRY(ctx, mlp_check_order(order, n, n_examples, d_flags, s), "index check kernel");
        PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 1, s));
        if (h_flags[0] != ~0ull) return set_error(ctx, PASTIS_E_INVAL, "order holds an index outside [0, n_examples)");
    }
    HIP_TRY(ctx, fill<uint32_t>((uint32_t *)lossd, nb, 0u, s), "reset");
    HIP_TRY(ctx, mlp_refresh(ctx->mlp, s), "refresh");
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t off = b * batch, cnt = std::min<int64_t>(batch, n - off);
        const int B = (int)((cnt + 15) / 16 * 16);
        HIP_TRY(ctx,
                mlp_batch_grad(ctx->mlp, X, labels, order, off, cnt, B, pos_weight, (float *)lossd + b, s),
                "gradient kernels");
        HIP_TRY(ctx, mlp_adam(ctx->mlp, lr, ++ctx->mlp_step, s), "adam kernel");
    }
    std::vector<float> h((size_t)nb);
    PASTIS_TRY(read_device(ctx, lossd, h.data(), sizeof(float) * nb, s));
    double acc = 0.0;
    for (float v : h) acc += v;
    if (mean_loss) *mean_loss = (float)(acc / (double)nb);
    return PASTIS_OK;
}

pastis_status pastis_mlp_calibrate(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n,
                                   double target_recall, float *tau, void *stream) {
    if (!ctx || n <= 0 || !X || !labels || !tau || !(target_recall > 0.0 && target_recall <= 1.0))
        return PASTIS_E_INVAL;
    PASTIS_TRY(need_net(ctx));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    void *logit = nullptr;
    PASTIS_TRY(ensure(ctx, kBufMlpLogit, sizeof(float) * (size_t)n, &logit));
    HIP_TRY(ctx, mlp_forward(ctx->mlp, X, n, (float *)logit, s), "network kernel");
    std::vector<float> y((size_t)n);
    std::vector<uint8_t> t((size_t)n);
    PASTIS_TRY(read_device(ctx, logit, y.data(), sizeof(float) * n, s));
    PASTIS_TRY(read_device(ctx, labels, t.data(), (size_t)n, s));
    std::vector<float> pos;
    for (int64_t q = 0; q < n; ++q)
        if (t[q]) pos.push_back(y[q]);
    if (pos.empty()) return set_error(ctx, PASTIS_E_INVAL, "no positive examples");
    std::sort(pos.begin(), pos.end());
    // keep logit >= tau for at least target_recall of the positives
    const size_t miss = (size_t)((1.0 - target_recall) * (double)pos.size());
    *tau = pos[std::min(miss, pos.size() - 1)];
    ctx->mlp_tau = *tau;
    return PASTIS_OK;
}

}  // extern "C"
