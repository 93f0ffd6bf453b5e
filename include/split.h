/*
 * split.h -- C ABI of the MI355X scenario-batched Split library (libsplitgpu.so).
 *
 * The operation (arXiv 2511.18022, Section 3, Eqs. (1)-(3)): a giant tour s_1..s_n is split
 * into capacity-feasible consecutive routes independently for every demand scenario w.
 * With f(0) = 0,
 *     f(i) = min over mask(i) <= p <= i-1 of
 *            f(p) + c(0, s_{p+1}) + sum_{k=p+1}^{i-1} c(s_k, s_{k+1}) + c(s_i, 0),
 *     mask(i) = smallest p < i with sum_{k=p+1}^{i} q^w_{s_k} <= Q            (Eq. (2)),
 * and the scenario's recourse cost is f(n). The expected second-stage cost of the tour is
 * the mean of f(n) over the scenarios (Section 2, two-stage objective; appendix, sample-
 * average problem). All cost and DP arithmetic is exact int32; demands are int16.
 *
 * Conventions used by every function:
 *  - Every function returns split_status; nothing throws, aborts, or prints.
 *  - Node 0 is the depot; customers are 1..N. The return depot of the paper (n+1) is the
 *    depot's location, so the closing arc of a route ending at customer c is d[c][0].
 *  - Unlimited fleet, no route-length limit (the optional limit the paper mentions is not used).
 *  - A context is not thread-safe: use one context per host thread / stream.
 *  - Limits: 1 <= n <= N <= SPLIT_MAX_N, Q >= 1 (any int32 capacity), 1 <= S < 2^31. The
 *    scenario-per-lane kernel compares load differences in 16 bits, exact while
 *    8 * max(q) + Q < 2^15; evaluations with Q > 16383 run in the wavefront-per-scenario form
 *    (exact for any Q) whatever form is chosen, and single scenarios outside the bound are
 *    handed to it. SPLIT_MAX_N is the wave kernel's LDS budget: it holds a scenario's prefix
 *    loads and DP values (8 bytes per position) in LDS.
 */
#ifndef SPLIT_H
#define SPLIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPLIT_MAX_N 8192

typedef enum {
    SPLIT_OK = 0,
    SPLIT_E_INVAL = -1,  /* NULL pointer, size out of range, ld < S, no instance set, ... */
    SPLIT_E_TOUR = -2,   /* a tour id outside 1..N, or repeated */
    SPLIT_E_DEMAND = -3, /* a scenario has a demand q < 0 or q > Q on the tour: Eq. (2)'s set
                            is empty, no feasible split exists (detected on the device) */
    SPLIT_E_RANGE = -4,  /* distances too large: the int32 DP could overflow */
    SPLIT_E_HIP = -5,    /* a HIP runtime call failed (message in split_last_error) */
    SPLIT_E_NOMEM = -6   /* device or host allocation failed */
} split_status;

/* Kernel form used by split_eval (all compute identical results). */
typedef enum {
    SPLIT_FORM_AUTO = 0, /* wavefront-per-scenario for short tours over few scenarios (n <= 32
                            at S <= 256, n <= 24 at S <= 1024, n <= 16 at S <= 4096),
                            scenario-per-lane otherwise */
    SPLIT_FORM_LANE = 1, /* one scenario per lane; sliding-window minimum in LDS (Q <= 16383;
                            a larger Q runs in the wave form) */
    SPLIT_FORM_WAVE = 2, /* one scenario per wavefront; lanes over predecessors p */
    SPLIT_FORM_MASK = 3  /* ablation, the two-kernel form of Section 3: the Eq. (2) window starts
                            of every state and scenario are written to an int16 matrix in device
                            memory (library-owned, 2 bytes per position and scenario), then a
                            second kernel scans each window (Eq. (3)). Not used by AUTO, the
                            autotuner or graphs. */
} split_form;

/*
 * Sample-average statistics of one split_eval call over its S scenarios.
 *  sum               = sum_s cost[s]                        (exact)
 *  sumsq_hi:sumsq_lo = sum_s cost[s]^2 as a 128-bit integer  (exact)
 *  mean = (double)sum / S
 *  var  = (((double)(S*sumsq - sum^2)) / S) / (S - 1)   sample variance, 0 when S == 1;
 *         the 128-bit numerator is exact and rounded to double once.
 *  n_fallback = scenarios whose capacity window outgrew the fast kernel's history and were
 *         re-evaluated by the general kernel (diagnostic only; results are exact either way).
 */
typedef struct {
    int64_t sum;
    uint64_t sumsq_lo;
    uint64_t sumsq_hi;
    double mean;
    double var;
    int64_t n_fallback;
} split_stats;

typedef struct split_ctx split_ctx;

/* Create a context on HIP device `hip_device`. *out receives the handle (NULL on failure). */
split_status split_ctx_create(int hip_device, split_ctx **out);

/* Free the context and its device buffers. Waits for the context's outstanding work. NULL ok. */
void split_ctx_destroy(split_ctx *ctx);

/* Human-readable message for the last failing call on ctx (valid until the next call). */
const char *split_last_error(const split_ctx *ctx);

/*
 * Set the instance from integer coordinates. xy: HOST, int32 [(N+1) * 2], node v at
 * (xy[2v], xy[2v+1]), node 0 the depot; |coordinate| <= 2^20. Distances are the Euclidean
 * distances rounded to the nearest integer (exact integer square root; halves cannot occur).
 * Copied; the caller keeps ownership. Errors: SPLIT_E_INVAL.
 */
split_status split_instance_set_coords(split_ctx *ctx, int32_t N, const int32_t *xy);

/*
 * Set the instance from a user distance matrix. d: HOST, int32 [(N+1) * (N+1)], row-major,
 * d[a*(N+1)+b] = cost of arc a->b (asymmetric allowed), all entries >= 0. Copied.
 * Errors: SPLIT_E_INVAL (N out of range, negative entry).
 */
split_status split_instance_set_dist(split_ctx *ctx, int32_t N, const int32_t *d);

/*
 * Evaluate one giant tour against S demand scenarios.
 *  tour   HOST int32 [n]: distinct customer ids in 1..N (a subset of the customers is allowed).
 *  demand DEVICE int16, N rows of leading dimension ld: demand[(c-1)*ld + s] is customer c's
 *         demand in scenario s (scenario index fastest). Read only.
 *  cost   DEVICE int32 [S]: receives f(n) for every scenario. Undefined on SPLIT_E_DEMAND.
 *  stats  HOST or NULL. Non-NULL: the call blocks until the statistics are on the host.
 *         NULL: the call only enqueues work on `hip_stream`; split_stats_get() collects the
 *         statistics (and any device-detected error) of the latest call later.
 *  hip_stream  hipStream_t to run on (NULL = the default stream).
 * The library never frees or retains caller pointers; enqueued work reads `demand` and
 * writes `cost` until the stream reaches it.
 * Errors: SPLIT_E_INVAL, SPLIT_E_TOUR, SPLIT_E_RANGE (4*(n+1)*max_arc >= 2^31),
 * SPLIT_E_DEMAND (blocking calls), SPLIT_E_HIP, SPLIT_E_NOMEM.
 */
split_status split_eval(split_ctx *ctx, const int32_t *tour, int32_t n, const int16_t *demand,
                        int64_t S, int64_t ld, int32_t Q, int32_t *cost, split_stats *stats,
                        void *hip_stream);

/*
 * split_eval for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same evaluation and results as
 * split_eval, with every per-call device buffer (the staged tour, the per-position arrays, the
 * result block, the counters and the moment partials) carved from a fixed scratch array of
 * 192 KiB that each GPU holds for the life of the process. The call makes no device or pinned
 * host allocation; the context, its instance and the caller's demand and cost buffers must
 * exist beforehand. Arguments as in split_eval; `tour` is copied from pageable host memory.
 *  stats  HOST or NULL. Non-NULL: the call waits for the evaluation and fills it. NULL: the
 *         call only enqueues (split_stats_get does not report these calls).
 * All calls on one GPU share its scratch, which keeps the last call's contents: calls that
 * overlap on one GPU (other streams, other host threads, other contexts) race; order them.
 * The context's timing and its latest-call statistics are left as they were.
 * Errors: as split_eval; SPLIT_E_INVAL also when the context's form is SPLIT_FORM_MASK (its
 * mask matrix needs an allocation) or a tour does not fit the scratch (never for n <= N <=
 * SPLIT_MAX_N).
 */
split_status split_eval_noalloc(split_ctx *ctx, const int32_t *tour, int32_t n,
                                const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                                int32_t *cost, split_stats *stats, void *hip_stream);

/*
 * Wait for the latest split_eval on ctx and return its statistics. Returns SPLIT_E_DEMAND if
 * that call found an infeasible demand, SPLIT_E_INVAL if no call was made yet.
 */
split_status split_stats_get(split_ctx *ctx, split_stats *stats);

/*
 * Evaluate T giant tours of uneven length against the same S demand scenarios in one launch
 * sequence: for every tour t, exactly what split_eval computes for it (Section 3, Eqs. (1)-(3);
 * the sample-average statistics of Section 2 and the appendix). The tours are the candidates a
 * search produces; the scenario matrix is read by all of them.
 *  tours     HOST int32, the T tours concatenated; tour t is tours[tour_ptr[t] .. tour_ptr[t+1]),
 *            distinct customer ids in 1..N within each tour (tours may share customers).
 *  tour_ptr  HOST int64 [T + 1], tour_ptr[0] = 0, every tour of length 1..N.
 *  demand    DEVICE int16 [N][ld] as in split_eval.
 *  cost      DEVICE int32 [T][ldc], ldc >= S: cost[t * ldc + s] receives f(n_t) of tour t in
 *            scenario s. Undefined for a tour whose status is SPLIT_E_DEMAND.
 *  stats     HOST [T] or NULL; tour_status HOST int32 [T] or NULL (per tour SPLIT_OK or
 *            SPLIT_E_DEMAND). If either is non-NULL the call blocks until both are filled; if
 *            both are NULL the call only enqueues work (split_batch_stats_get collects them).
 * Work items are scheduled as the context's launch choices say (split_tuning). The library
 * copies the tours; enqueued work reads `demand` and writes `cost` until the stream reaches it.
 * Errors: as split_eval (SPLIT_E_TOUR names the tour), SPLIT_E_INVAL also when
 * T * ceil(S / 64) >= 2^31; SPLIT_E_DEMAND when some tour's status is SPLIT_E_DEMAND.
 */
split_status split_eval_batch(split_ctx *ctx, const int32_t *tours, const int64_t *tour_ptr,
                              int32_t T, const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                              int32_t *cost, int64_t ldc, split_stats *stats,
                              int32_t *tour_status, void *hip_stream);

/*
 * Wait for the latest evaluation on ctx (split_eval counts as a batch of one) and fill
 * stats[0 .. T-1] and tour_status[0 .. T-1] (either may be NULL). Returns SPLIT_E_DEMAND if
 * some tour's status is SPLIT_E_DEMAND, SPLIT_E_INVAL if no call was made yet.
 */
split_status split_batch_stats_get(split_ctx *ctx, split_stats *stats, int32_t *tour_status);

/* Choose the kernel form for later split_eval calls (default SPLIT_FORM_AUTO). */
split_status split_set_form(split_ctx *ctx, int form);

/*
 * Launch choices of the evaluations (none changes a result: every choice computes exactly
 * Section 3's Eqs. (1)-(3)).
 *  form         split_form; SPLIT_FORM_AUTO takes the wave form for short tours over few
 *               scenarios (see split_form), else the lane form.
 *  lane_per_cu  lane form: 0 = the library's choice: over one tour whose work items (64 of
 *               its scenarios each) are at most 16 per workgroup, 8 persistent workgroups per
 *               compute unit, each taking work items at a fixed stride; otherwise one
 *               workgroup per work item. 1..8 = that many persistent workgroups per compute
 *               unit, taking work items from a queue.
 *  order        lane form: 0 = work items of longer tours first, 1 = tours in the given order.
 *  wave_grid    wave form: workgroups of the launch; 0 = min(T * S, 65536).
 *  lane_block   lane form: states per block of the scenario-per-lane kernel, 0 or 16 = 16,
 *               or 8. A block's windows (Eq. (3)) are looked up in O(1) while they start
 *               before the block; 16 suits windows of about 16..47 positions, 8 shorter ones
 *               (about 8..23 positions; Q / mean demand estimates the window). Scenarios whose
 *               windows outgrow three blocks are finished exactly by the wave kernel either way.
 * The default is {SPLIT_FORM_AUTO, 0, 0, 0, 0}. split_set_form sets `form` alone.
 */
typedef struct {
    int32_t form;
    int32_t lane_per_cu;
    int32_t order;
    int32_t wave_grid;
    int32_t lane_block;
} split_tuning;

/* Set / read the context's launch choices. Errors: SPLIT_E_INVAL (a field out of range). */
split_status split_tuning_set(split_ctx *ctx, const split_tuning *tuning);
split_status split_tuning_get(split_ctx *ctx, split_tuning *tuning);

/*
 * Autotuner: times whole evaluations (tour upload, kernels, statistics; HIP events on
 * hip_stream, `reps` timed calls after one warm-up each) of this batch under the candidate
 * launch choices, installs the fastest in the context and returns it with its mean
 * milliseconds (either output may be NULL). Candidates: lane form with lane_block 16 and 8
 * (lane_per_cu 0, order 0; 8 only when, over the first 4096 scenarios, it leaves no more
 * scenarios to the wave kernel than 16 does), then lane_per_cu in {0, 8, 4, 2} and both orders
 * with the faster block length; wave form with wave_grid in {0, 8 per CU} when a run on 256
 * scenarios, scaled to S, comes within 1.5x of the best lane time. Arguments as in
 * split_eval_batch; `cost` is overwritten and ends holding the batch's costs under the chosen
 * tuning, and the context's latest evaluation (split_batch_stats_get) is that one.
 * Blocks until done. Errors: as split_eval_batch; SPLIT_E_INVAL if reps is not in 1..1000.
 * The context's tuning is unchanged on error.
 */
split_status split_autotune(split_ctx *ctx, const int32_t *tours, const int64_t *tour_ptr,
                            int32_t T, const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                            int32_t *cost, int64_t ldc, int32_t reps, void *hip_stream,
                            split_tuning *best, double *best_ms);

/*
 * Captured evaluation: the whole split_eval_batch sequence (tour upload from pinned host
 * memory, prep, Split DP, moments, statistics copy) recorded once as a HIP graph for a fixed
 * demand matrix, cost matrix, S, Q and instance, then replayed with new tours by
 * split_graph_launch: one graph launch per batch, for search loops that evaluate many batches.
 * Results are exactly those of split_eval_batch (Section 3, Eqs. (1)-(3)).
 *  max_T, max_total_n  capacity: at most max_T tours and max_total_n positions per launch.
 *  demand    DEVICE int16 [N][ld] holding a row for every customer 1..N of the instance.
 *  cost      DEVICE int32 [max_T][ldc]; each launch writes rows 0..T-1.
 * The graph copies the context's instance and launch choices at creation (later changes to the
 * context do not reach it) and owns its device buffers; demand and cost stay the caller's and
 * must outlive the graph. Launches of one graph must be ordered (one stream, or synchronized).
 * Errors: as split_eval_batch for the shapes; SPLIT_E_INVAL for a capacity out of range
 * (1 <= max_T <= max_total_n <= max_T * N, max_T * ceil(S / 64) < 2^31); SPLIT_E_RANGE when
 * 4 * (N + 1) * max_arc >= 2^31; SPLIT_E_HIP when capture or instantiation fails.
 */
typedef struct split_graph split_graph;
split_status split_graph_create(split_ctx *ctx, int32_t max_T, int64_t max_total_n,
                                const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                                int32_t *cost, int64_t ldc, split_graph **out);

/*
 * Stage T tours (HOST arrays as in split_eval_batch; copied into the graph's pinned memory,
 * after waiting for the launch before the previous one to finish with it) and launch the
 * graph on hip_stream. Errors: SPLIT_E_INVAL (T or the positions over capacity, a bad tour
 * length), SPLIT_E_TOUR, SPLIT_E_RANGE, SPLIT_E_HIP. Error messages go to the creating context.
 */
split_status split_graph_launch(split_graph *graph, const int32_t *tours,
                                const int64_t *tour_ptr, int32_t T, void *hip_stream);

/*
 * Wait for the graph's latest launch and fill stats[0..T-1] and tour_status[0..T-1] (either may
 * be NULL), as split_batch_stats_get. Returns SPLIT_E_DEMAND if some tour's status is.
 */
split_status split_graph_stats(split_graph *graph, split_stats *stats, int32_t *tour_status);

/* Wait for the graph's launches and free it. NULL ok. Destroy graphs before their context. */
void split_graph_destroy(split_graph *graph);

/*
 * Kernel timing for benchmarks: when enabled, split_eval records HIP events around its
 * dominant kernel on the caller's stream. split_timing_get waits for the last call and
 * returns the accumulated dominant-kernel milliseconds and the number of timed launches
 * since the last reset, with the name of the kernel timed.
 */
split_status split_timing_enable(split_ctx *ctx, int enable);
split_status split_timing_get(split_ctx *ctx, double *ms_total, int64_t *launches,
                              const char **kernel_name);
split_status split_timing_reset(split_ctx *ctx);
/* The duration of every timed launch since the last reset, in order: ms HOST float [cap]
 * receives the first min(cap, *count) of them (ms may be NULL when cap is 0); *count receives
 * how many there are. Waits for the last call. */
split_status split_timing_samples(split_ctx *ctx, float *ms, int64_t cap, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* SPLIT_H */
