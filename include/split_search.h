/*
 * split_search.h -- C ABI of the local search in libsplitgpu.so.
 *
 * A small search loop over giant tours that uses the scenario-batched Split as its objective:
 * the expected second-stage cost of a tour, i.e. the mean over the scenarios of f(n) from
 * arXiv 2511.18022, Section 3, Eqs. (1)-(3) (Section 2's sample-average objective). It mirrors
 * the role the paper gives fast Split evaluation inside a search under a time budget (the
 * quality-over-time experiment of Section 4), with a plain neighbourhood search instead of the
 * paper's genetic search.
 *
 * Iteration: `pool` neighbours of the incumbent are drawn (each a 2-opt move -- reverse
 * positions i..j -- or a relocate move -- take the customer at position i out and insert it at
 * position j -- with equal probability, i != j uniform, from a splitmix64 stream of `seed`).
 * Without a surrogate (nn == NULL) pool must equal batch and all of them are evaluated exactly.
 * With a surrogate the pool is built on the device from the incumbent and the moves, predicted,
 * and the `batch` lowest predictions are evaluated exactly (split_nn_shortlist; ties go to the
 * earlier drawn move). Exact evaluation replays a captured graph
 * (split_graph_*). The incumbent moves to the best evaluated neighbour when its exact mean is
 * lower. The loop stops when budget_s seconds of wall-clock time have passed (checked after
 * every iteration) or after max_iters iterations.
 */
#ifndef SPLIT_SEARCH_H
#define SPLIT_SEARCH_H

#include <stdint.h>

#include "split.h"
#include "split_nn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t iterations;   /* iterations run */
    int64_t evaluated;    /* tours evaluated exactly (the start tour included) */
    int64_t predicted;    /* tours scored by the surrogate */
    int64_t improvements; /* accepted moves */
    double start_mean;    /* exact mean of the start tour */
    double best_mean;     /* exact mean of the returned tour */
    double seconds;       /* wall-clock time of the search */
} split_search_result;

/*
 * tour0      HOST int32 [n]: the start tour (distinct customer ids 1..N).
 * demand     DEVICE int16 [N][ld] with a row for every customer of the instance; S, Q as in
 *            split_eval.
 * batch      tours evaluated exactly per iteration (1..4096); pool >= batch (== batch when
 *            nn is NULL), pool <= 65536.
 * best_tour  HOST int32 [n]: receives the best tour found.
 * trace_t, trace_mean  HOST double [trace_cap] or NULL: (seconds, exact mean) of the start tour
 *            and of every accepted move, in order; *trace_len receives the count (at most
 *            trace_cap are written).
 * Blocks. Errors: SPLIT_E_INVAL (sizes, no instance), SPLIT_E_TOUR, SPLIT_E_DEMAND (some
 * scenario infeasible on the tour), SPLIT_E_RANGE, SPLIT_E_HIP, SPLIT_E_NOMEM.
 */
split_status split_search(split_ctx *ctx, split_nn *nn, const int32_t *tour0, int32_t n,
                          const int16_t *demand, int64_t S, int64_t ld, int32_t Q, int32_t batch,
                          int32_t pool, double budget_s, int64_t max_iters, uint64_t seed,
                          int32_t *best_tour, double *trace_t, double *trace_mean,
                          int32_t trace_cap, int32_t *trace_len, split_search_result *result,
                          void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SPLIT_SEARCH_H */
