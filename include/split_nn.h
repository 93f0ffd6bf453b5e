/*
 * split_nn.h -- C ABI of the tour-encoder surrogate in libsplitgpu.so.
 *
 * The surrogate is not part of arXiv 2511.18022. It predicts a giant tour's expected
 * second-stage cost -- the sample mean over the scenarios of the Split cost f(n) that Section 3
 * (Eqs. (1)-(3)) computes and split_eval returns -- so that a search can rank many candidate
 * tours cheaply and re-evaluate only a shortlist exactly with split_eval_batch.
 *
 * Network (bf16 weights and activations, fp32 accumulation, fp32 master weights):
 *   features of tour position j (s_0 = s_{n+1} = depot 0; L = length scale, Q = capacity):
 *     (x(s_j) - x(0)) / L, (y(s_j) - y(0)) / L   (0 for an instance given as a matrix)
 *     mean(q_{s_j}) / Q, std(q_{s_j}) / Q        (over the scenarios; population std)
 *     c(s_{j-1}, s_j) / L, c(s_j, s_{j+1}) / L, c(0, s_j) / L, 1
 *   H_l = relu(conv_l(H_{l-1}) + b_l), l = 1..4, 5 taps, 128 channels, zero padding, where
 *     conv(H)[j] = sum_{k=0..4} H[j + k - 2] . W[k]  (cross-correlation, same length)
 *   z = mean_j H_4[j]; u = relu(Wa z + ba); y = wb . u + bb; prediction = y * scale + shift.
 * Training minimizes the mean over a batch of (y - (label - shift) / scale)^2 with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Flat fp32 parameter vector (SPLIT_NN_PARAMS values, in this order):
 *   W1 [5][32][128] (only input channels 0..7 meet nonzero features), b1 [128],
 *   W2, W3, W4 [5][128][128] each followed by its bias [128],
 *   Wa [128][128] (row = output unit), ba [128], wb [128], bb [1].
 *
 * Conventions: as split.h. Tours passed to these functions are DEVICE int32 [T][n] (every tour
 * of one call has the same length n, ids 1..N of the context's instance, distinct within a
 * tour); an id out of range makes the call fail with SPLIT_E_TOUR. Every reduction runs in a
 * fixed order, so results are bitwise reproducible for the same inputs.
 */
#ifndef SPLIT_NN_H
#define SPLIT_NN_H

#include <stdint.h>

#include "split.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SPLIT_NN_PARAMS 283393

typedef struct split_nn split_nn;

/*
 * A surrogate on ctx's device, using ctx's instance (set before the first call that needs
 * features). Parameters: He-uniform conv and MLP weights from `seed`, zero biases; Adam state
 * zero; normalization shift 0, scale 1. length_scale > 0 divides coordinates and arc costs.
 * Destroy surrogates before their context.
 */
split_status split_nn_create(split_ctx *ctx, uint64_t seed, double length_scale, split_nn **out);
void split_nn_destroy(split_nn *nn);

/* HOST fp32 [SPLIT_NN_PARAMS] in the order above. set also resets the Adam state and step. */
split_status split_nn_params_get(split_nn *nn, float *params);
split_status split_nn_params_set(split_nn *nn, const float *params);

/* prediction = y * scale + shift (scale > 0). */
split_status split_nn_set_norm(split_nn *nn, double shift, double scale);

/*
 * The scenario set the demand features come from: DEVICE int16 [N][ld] as in split_eval, its
 * first S scenarios, capacity Q. Computes every customer's demand mean and std on the device.
 */
split_status split_nn_set_scenarios(split_nn *nn, const int16_t *demand, int64_t S, int64_t ld,
                                    int32_t Q);

/* Predicted expected cost of T tours: pred DEVICE fp32 [T]. Enqueued on hip_stream; blocks
 * only to check the tour ids. */
split_status split_nn_predict(split_nn *nn, const int32_t *tours, int32_t T, int32_t n,
                              float *pred, void *hip_stream);

/*
 * Loss and gradient of one batch without updating: labels DEVICE fp32 [T] (expected costs),
 * grad HOST fp32 [SPLIT_NN_PARAMS] or NULL, loss HOST or NULL (the batch MSE in normalized
 * units). Blocks.
 */
split_status split_nn_gradient(split_nn *nn, const int32_t *tours, const float *labels,
                               int32_t T, int32_t n, float *grad, double *loss, void *hip_stream);

/* One Adam step on one batch (the gradient of split_nn_gradient), learning rate lr. loss HOST or
 * NULL: if non-NULL the call blocks and returns the batch loss before the update. */
split_status split_nn_train_step(split_nn *nn, const int32_t *tours, const float *labels,
                                 int32_t T, int32_t n, float lr, double *loss,
                                 void *hip_stream);

/*
 * `steps` Adam steps over a training set of `count` tours (DEVICE int32 [count][n], labels
 * DEVICE fp32 [count]) in batches of `batch`: global step b uses batch b mod (count / batch) of
 * the permutation of epoch b / (count / batch), drawn from `seed`. The run starts at the
 * surrogate's step counter, so a run split by split_nn_save / split_nn_load is bitwise the
 * same as one run. mean_loss HOST or NULL: mean batch loss of the run's steps. Blocks.
 */
split_status split_nn_train(split_nn *nn, const int32_t *tours, const float *labels,
                            int64_t count, int32_t n, int32_t batch, int64_t steps, float lr,
                            uint64_t seed, double *mean_loss, void *hip_stream);

/* Step counter (Adam steps taken). */
split_status split_nn_step(split_nn *nn, int64_t *step);

/*
 * Checkpoint: parameters, Adam moments, step counter, normalization and length scale in one
 * binary file (little-endian, magic "SPLITNN1"). load requires a file of this layout.
 * Errors: SPLIT_E_INVAL (unreadable or foreign file).
 */
split_status split_nn_save(split_nn *nn, const char *path);
split_status split_nn_load(split_nn *nn, const char *path);

/*
 * Indices of the K smallest of C scores (DEVICE fp32 [C]) into idx DEVICE int32 [K], in
 * increasing index order; ties at the threshold go to the lower indices. 1 <= K <= C < 2^31.
 */
split_status split_topk_smallest(split_ctx *ctx, const float *scores, int64_t C, int64_t K,
                                 int32_t *idx, void *hip_stream);

/*
 * Predict T tours (DEVICE int32 [T][n]) and write the indices of the K lowest predictions to
 * idx (DEVICE int32 [K], increasing; ties to the lower index), using the surrogate's own
 * scratch. pred DEVICE fp32 [T] or NULL (then internal). Blocks. 1 <= K <= T.
 */
split_status split_nn_shortlist(split_nn *nn, const int32_t *tours, int32_t T, int32_t n,
                                int32_t K, int32_t *idx, float *pred, void *hip_stream);

/*
 * Screening: predict the C candidate tours (DEVICE int32 [C][n]), keep the K with the lowest
 * prediction, evaluate those exactly with split_eval_batch against demand (DEVICE int16
 * [N][ld], S scenarios, capacity Q), and return the best by exact mean.
 *  pred       DEVICE fp32 [C] or NULL: receives the predictions.
 *  short_idx  HOST int32 [K] or NULL: the shortlist (candidate indices, increasing).
 *  short_mean HOST double [K] or NULL: their exact means.
 *  best_idx, best_mean  HOST: the best shortlisted candidate (lowest exact mean; lowest index
 *             on ties) and its exact mean.
 * Blocks. Errors: as split_nn_predict and split_eval_batch.
 */
split_status split_nn_screen(split_nn *nn, const int32_t *cands, int64_t C, int32_t n, int64_t K,
                             const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                             float *pred, int32_t *short_idx, double *short_mean,
                             int64_t *best_idx, double *best_mean, void *hip_stream);

/*
 * Kernel timing for benchmarks: when enabled, every prediction records HIP events on the
 * caller's stream around the fused convolution kernel (the four conv layers and the pooling,
 * one launch per forward pass of up to 1024 tours). split_nn_timing_get waits for the recorded
 * launches and returns their accumulated milliseconds and count since the last reset.
 */
split_status split_nn_timing_enable(split_nn *nn, int enable);
split_status split_nn_timing_get(split_nn *nn, double *ms_total, int64_t *launches);
split_status split_nn_timing_reset(split_nn *nn);

#ifdef __cplusplus
}
#endif

#endif /* SPLIT_NN_H */
