// Internal interface between the surrogate's host layer (nn_host.cpp) and its HIP kernels
// (nn_kernels.hip). Not installed; callers use include/split_nn.h.
//
// Flat fp32 parameter vector (the order of split_nn.h):
//   W1 [5][32][128], b1 [128], W2 [5][128][128], b2, W3, b3, W4, b4,
//   Wa [128][128] (row = output), ba [128], wb [128], bb [1]
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace splitgpu {

constexpr int kNnTaps = 5;
constexpr int kNnCi0 = 32;     // input channels of layer 1 (8 features, zero-padded)
constexpr int kNnFeatures = 8;  // the features: channels 0..7 of layer 1's input
constexpr int kNnWidth = 128;  // channels of every conv layer and of the MLP

constexpr int kNnSizeW1 = kNnTaps * kNnCi0 * kNnWidth;
constexpr int kNnSizeWl = kNnTaps * kNnWidth * kNnWidth;
__host__ __device__ constexpr int nn_off_w(int l)  // l = 0..3 for W1..W4
{
    return l == 0 ? 0 : kNnSizeW1 + kNnWidth + (l - 1) * (kNnSizeWl + kNnWidth);
}
__host__ __device__ constexpr int nn_off_b(int l) { return nn_off_w(l) + (l == 0 ? kNnSizeW1 : kNnSizeWl); }
constexpr int kNnOffWa = nn_off_b(3) + kNnWidth;
constexpr int kNnOffBa = kNnOffWa + kNnWidth * kNnWidth;
constexpr int kNnOffWb = kNnOffBa + kNnWidth;
constexpr int kNnOffBb = kNnOffWb + kNnWidth;
constexpr int kNnParams = kNnOffBb + 1;
static_assert(kNnParams == 283393, "parameter layout");

// The instance as the feature kernel reads it.
struct NnInstance {
    int32_t N;
    int32_t kind;         // 0 coordinates, 1 distance matrix
    const int32_t *xy;    // device [(N+1)*2]
    const int32_t *dist;  // device [(N+1)^2]
};

// bf16 weight copies: f[l] = forward layout [co][tap * CI + ci]; b[l] (l >= 1) = backward-data
// layout [ci][tap' * 128 + co] with tap' = 4 - tap.
struct NnWeights {
    uint16_t *f[4];  // layer l: bf16 [co][tap * CI + ci]
    uint16_t *b[4];  // layers 1..3: the flipped, transposed taps for the data gradient
    uint16_t *g[4];  // layer l in MFMA fragment order (the fused prediction kernel's reads)
};

// Radix-select state: the key prefix found so far, its mask, and the rank still to reach.
struct NnSelect {
    uint32_t prefix;
    uint32_t mask;
    unsigned long long rank;
};

hipError_t nn_launch_dstats(const int16_t *demand, int64_t ld, int64_t S, int32_t N, double *musd,
                            hipStream_t st);
// the 8 bf16 features of every position: packed [T][n][8] for prediction, else the padded
// training layout [T][n + 4][32] (rows 0, 1, n + 2, n + 3 and channels 8..31 left untouched)
hipError_t nn_launch_features(const NnInstance &in, const int32_t *tours, int32_t T, int32_t n,
                              const double *musd, int32_t Q, double L, uint16_t *X, bool packed,
                              int32_t *err, hipStream_t st);
hipError_t nn_launch_conv(int ci, int mode, const uint16_t *X, const uint16_t *Wt,
                          const float *bias, const uint16_t *mask, uint16_t *Y, int32_t T,
                          int32_t n, hipStream_t st);
// prediction only: the four conv layers per tile in LDS, pooled into per-tile channel sums
// (zpart [T][tiles][128]) from the packed features X [T][n][8]; then the pooled mean and the head
int32_t nn_fused_tiles(int32_t n);
hipError_t nn_launch_fwd_fused(const uint16_t *X, const NnWeights &w, const float *P, int32_t T,
                               int32_t n, float *zpart, hipStream_t st);
hipError_t nn_launch_head_pool(const float *zpart, int32_t T, int32_t n, const float *P, float *z,
                               float *a, float *y, float *pred, double shift, double scale,
                               hipStream_t st);
hipError_t nn_launch_head_fwd(const uint16_t *H4, int32_t T, int32_t n, const float *P, float *z,
                              float *a, float *y, float *pred, double shift, double scale,
                              hipStream_t st);
hipError_t nn_launch_head_bwd(const float *labels, int32_t T, int32_t n, const float *P,
                              const float *z, const float *a, const float *y, double shift,
                              double scale, float *da, float *dz, float *dy, float *loss_terms,
                              const uint16_t *H4, uint16_t *dP4, float *G, hipStream_t st);
// number of weight-gradient partials for a batch: chunks of `chunk` padded rows
int32_t nn_wgrad_chunks(int32_t T, int32_t n, int32_t chunk);
hipError_t nn_launch_wgrad(int ci, const uint16_t *H, const uint16_t *dP, int32_t T, int32_t n,
                           int32_t chunk, int32_t chunks, float *partW, float *partB, float *G,
                           int32_t offW, int32_t offB, hipStream_t st);
hipError_t nn_launch_adam(float *P, float *m, float *v, const float *G, float lr, float bc1,
                          float bc2, hipStream_t st);
hipError_t nn_launch_pack(const float *P, const NnWeights &w, hipStream_t st);
hipError_t nn_launch_gather(const int32_t *src, const float *lab, const int32_t *idx, int32_t B,
                            int32_t n, int32_t *dst, float *dlab, hipStream_t st);
hipError_t nn_launch_loss(const float *terms, int32_t T, float *out, hipStream_t st);
// candidates [count][n] from cur [n] and moves [count][3] = (type, i, j), validated by the caller
hipError_t nn_launch_moves(const int32_t *cur, const int32_t *moves, int32_t count, int32_t n,
                           int32_t *out, hipStream_t st);
hipError_t nn_launch_check_ids(const int32_t *ids, long long count, int32_t N, int32_t *err,
                               hipStream_t st);
hipError_t nn_launch_topk(const float *s, long long C, long long K, NnSelect *sel,
                          unsigned long long *hist, unsigned int *cnt, unsigned long long *base,
                          int32_t *idx, hipStream_t st);

}  // namespace splitgpu
