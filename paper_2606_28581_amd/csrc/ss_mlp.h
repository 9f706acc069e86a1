// Internal declarations of the surrogate MLP kernels (layout constants, launchers).
#pragma once
#include "ss_internal.h"

namespace ss {

constexpr int kMlpIn = 128, kMlpWidth = 64;
constexpr int kMlpW1 = kMlpWidth * kMlpIn, kMlpW2 = kMlpWidth * kMlpWidth, kMlpW3 = kMlpW2;
// offsets in the FP32 master parameter vector [W1, b1, W2, b2, W3, b3, w4, b4]
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpW1, kOffW2 = kOffB1 + kMlpWidth;
constexpr int kOffB2 = kOffW2 + kMlpW2, kOffW3 = kOffB2 + kMlpWidth;
constexpr int kOffB3 = kOffW3 + kMlpW3, kOffW4 = kOffB3 + kMlpWidth, kOffB4 = kOffW4 + kMlpWidth;
constexpr int kMlpParams = kOffB4 + 1;   // 16641
constexpr int kMlpBf16 = kMlpW1 + kMlpW2 + kMlpW3 + kMlpWidth;
constexpr int kMlpF32 = 3 * kMlpWidth + 1;
constexpr int kDwChunk = 512;            // points per block in the weight-gradient kernels

struct MlpNorm {
    float cx, cy, cz, inv_half;
};

int mlp_dw_blocks(int64_t M);
hipError_t launch_mlp_prep(const float *w, uint16_t *wb, float *wf, hipStream_t st);
// logits[i] (or sigmoid(logit) when `prob`) for points i < M; G > 0: position i % G,
// sun i / G; G == 0: position i, sun i.  saveF [M,128], saveH [3][M,64] bf16 or NULL.
hipError_t launch_mlp_forward(const uint16_t *wb, const float *wf, const float *pts,
                              const float *sun, int64_t M, int64_t G, MlpNorm nz, bool prob,
                              float *out, uint16_t *saveF, uint16_t *saveH, hipStream_t st);
// dlogit = labels ? (sigmoid(logit) - y) * scale : dlogit_in * scale; da3 = bf16(dlogit w4
// [h3 > 0]); partial sums of dw4 (64), db4 and the BCE loss per block.
hipError_t launch_mlp_out_bwd(const float *logits, const float *labels, const float *dlogit_in,
                              float scale, const uint16_t *wb, const uint16_t *H3, int64_t M,
                              uint16_t *dA3, float *part, hipStream_t st);
// part_dw[blk][64][n] = sum over the block's points of dA[m][i] H[m][j];
// part_db[blk][64] = sum of dA[m][i]
hipError_t launch_mlp_dw(const uint16_t *dA, const uint16_t *H, int n, int64_t M,
                         float *part_dw, float *part_db, hipStream_t st);
// dA_prev[m][j] = bf16((dA W)[m][j] * [Hprev[m][j] > 0]),  W = 64x64 bf16 of a layer
hipError_t launch_mlp_dh(const uint16_t *dA, const uint16_t *Wb, const uint16_t *Hprev,
                         int64_t M, uint16_t *dA_prev, hipStream_t st);
// grad[offset ...] = sum over blocks of part[blk][count]
hipError_t launch_mlp_reduce(const float *part, int nblocks, int count, int stride, float *out,
                             hipStream_t st);
hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr,
                           float b1, float b2, float eps, int step, hipStream_t st);

}  // namespace ss
