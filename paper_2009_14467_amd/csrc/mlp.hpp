// Learned pre-alignment filter (see mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pastis {

constexpr int kMlpIn = 16, kMlpHidden = 128;
// flat fp32 parameter vector: W1 [128][16], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]
constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpHidden * kMlpIn;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpHidden;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpHidden * kMlpHidden;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpHidden;
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpHidden;
constexpr int kMlpParams = kMlpOffB3 + 1;
// per-block partial sums of one training minibatch: loss, b1, b2, w3, b3;
// a training block holds kMlpTrainWaves waves of 16 pairs each
constexpr int kMlpPartN = 1 + 3 * kMlpHidden + 1;
constexpr int kMlpTrainWaves = 4;
// the weight-gradient reductions over a minibatch are split into chunks of
// this many pairs, one wave per (output tile, chunk)
constexpr int kMlpSplitK = 256;

// Device state of the network (owned by the context).
struct MlpState {
    float *theta, *m, *v, *grad;           // kMlpParams each
    uint16_t *W1b, *W2b, *W2Tb, *w3b;      // bf16 copies
    float *mean, *stdv;                    // kMlpIn each
    double *moments;                       // 2 * kMlpIn
    uint16_t *ZT, *H1, *DH2, *DH1;         // per-batch activations, feature-major
    int batch_cap;                         // pairs the activation buffers hold
    float *part;                           // [batch_cap / (16 * kMlpTrainWaves)][kMlpPartN] block partials
    float *wpart;                          // [batch_cap / kMlpSplitK][W2 then W1] chunk partials
    // labelled examples collected for training: features [pool_cap][16], labels
    float *pool_X = nullptr;
    uint8_t *pool_y = nullptr;
    int64_t pool_n = 0, pool_cap = 0;
};

hipError_t mlp_refresh(const MlpState &S, hipStream_t s);
hipError_t mlp_features(const uint8_t *codes, const int64_t *offsets, int64_t n, const uint32_t *lo,
                        const uint32_t *hi, const uint32_t *count, const uint32_t *s1, const uint32_t *s2,
                        int64_t npairs, float *comp, float *F, hipStream_t s);
hipError_t mlp_forward(const MlpState &S, const float *X, int64_t n, float *logits, hipStream_t s);
hipError_t mlp_moments(const float *X, int64_t n, double *acc, float *mean, float *stdv, hipStream_t s);
// Gradient of the weighted logistic loss over examples order[off .. off +
// count) (B = count rounded up to 16) into S.grad, the batch loss added to
// *loss; step > 0 also takes Adam step number `step` at learning rate lr.
// The sums run in a fixed order: the same inputs give the same bits.
hipError_t mlp_batch_grad(const MlpState &S, const float *X, const uint8_t *labels, const int32_t *order, int64_t off,
                          int64_t count, int B, float pos_weight, float *loss, float lr, int step, hipStream_t s);
hipError_t mlp_keep(const float *logits, int64_t n, float tau, uint8_t *keep, hipStream_t s);
hipError_t mlp_check_order(const int32_t *order, int64_t n, int64_t limit, unsigned long long *flag, hipStream_t s);
hipError_t compact5(const uint8_t *keep, const uint32_t *pos, int64_t n, const uint32_t *const in[5],
                    uint32_t *const out[5], hipStream_t s);

}  // namespace pastis
