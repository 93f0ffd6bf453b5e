/*
 * CPU oracle for the scenario-batched Split (arXiv 2511.18022, "GPU-based Split algorithm
 * for Large-Scale CVRPSD").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct reference that
 * the GPU library is checked against. Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load it; the GPU library never calls, links or includes
 * it, and it includes nothing from the GPU library.
 *
 * What it computes, by section of the paper:
 *  - Section 3, Eq. (1): for every scenario w, f(0) = 0 and
 *      f(i) = min over 0 <= p <= i-1 of  f(p) + c(0, s_{p+1}) + sum_{k=p+1}^{i-1} c(s_k, s_{k+1})
 *                                         + c(s_i, n+1)
 *    subject to  sum_{k=p+1}^{i} q_{s_k} <= Q ;  the scenario's recourse cost is f(n).
 *    The return depot n+1 is the depot's location: c(s_i, n+1) = d[s_i][0].
 *  - Section 3, Eq. (2): mask(i) = smallest p in [0, i) with sum_{k=p+1}^{i} q_{s_k} <= Q.
 *  - Section 3, Eq. (3): the same minimum taken over p in [mask(i), i-1] with no test.
 *  - Section 2 (two-stage objective) and the appendix (sample-average problem): the
 *    expected second-stage cost is the plain mean of f(n) over the scenarios.
 *  - Distances (not specified by the paper): nearest integer of the Euclidean distance
 *    between integer coordinates, computed exactly with an integer square root.
 *
 * Readings where the paper is silent: demands must satisfy 0 <= q <= Q (a larger demand
 * leaves Eq. (2)'s set empty and the scenario has no feasible split: status -3); the fleet
 * is unlimited; no route-length limit; the variance is the sample variance (denominator
 * S - 1, 0 when S = 1) computed from exact integer moments.
 *
 * The one liberty taken with Eq. (1): the candidates p are visited from i-1 downwards and the
 * scan stops at the first p whose segment load exceeds Q. With demands >= 0 the segment load
 * only grows as p decreases, so every smaller p is infeasible too; the result is unchanged.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_TOUR (-2)
#define OR_E_DEMAND (-3)
#define OR_E_NOMEM (-6)

/* floor(sqrt(m)) for 0 <= m < 2^62, by the classic bit-by-bit method (no floating point). */
int64_t or_isqrt(int64_t m)
{
    if (m <= 0) return 0;
    uint64_t x = (uint64_t)m, r = 0, bit = (uint64_t)1 << 62;
    while (bit > x) bit >>= 2;
    while (bit) {
        if (x >= r + bit) {
            x -= r + bit;
            r = (r >> 1) + bit;
        } else {
            r >>= 1;
        }
        bit >>= 2;
    }
    return (int64_t)r;
}

/* Nearest integer to sqrt(dx^2 + dy^2): k = isqrt(m); round up iff m > k^2 + k, because
 * (k + 1/2)^2 = k^2 + k + 1/4 and m is an integer (so no exact halves occur). */
int64_t or_nint_dist(int64_t x1, int64_t y1, int64_t x2, int64_t y2)
{
    int64_t dx = x1 - x2, dy = y1 - y2;
    int64_t m = dx * dx + dy * dy;
    int64_t k = or_isqrt(m);
    return (m > k * k + k) ? k + 1 : k;
}

/* Full (N+1) x (N+1) distance matrix from coordinates xy[2*(N+1)]; node 0 is the depot. */
int or_dist_from_coords(int32_t N, const int32_t *xy, int32_t *d)
{
    if (N < 1 || !xy || !d) return OR_E_INVAL;
    int64_t V = (int64_t)N + 1;
    for (int64_t a = 0; a < V; ++a)
        for (int64_t b = 0; b < V; ++b) {
            int64_t v = or_nint_dist(xy[2 * a], xy[2 * a + 1], xy[2 * b], xy[2 * b + 1]);
            if (v > INT32_MAX) return OR_E_INVAL;
            d[a * V + b] = (int32_t)v;
        }
    return OR_OK;
}

/* Tour check: ids in 1..N, pairwise distinct. */
static int check_tour(const int32_t *tour, int32_t n, int32_t N)
{
    char *seen = (char *)calloc((size_t)N + 1, 1);
    if (!seen) return OR_E_NOMEM;
    int rc = OR_OK;
    for (int32_t k = 0; k < n; ++k) {
        int32_t c = tour[k];
        if (c < 1 || c > N || seen[c]) {
            rc = OR_E_TOUR;
            break;
        }
        seen[c] = 1;
    }
    free(seen);
    return rc;
}

#define DIST(a, b) ((int64_t)d[(int64_t)(a) * V + (b)])

/*
 * Eq. (1) for one scenario. q[k] is the demand of the customer at tour position k+1
 * (already gathered), f is scratch of n+1 entries. Returns the cost through *cost and adds
 * the number of feasible transitions beyond the first, sum_i (w_i - 1), to *work.
 */
static int split_one(const int32_t *tour, int32_t n, const int32_t *d, int64_t V,
                     const int32_t *q, int32_t Q, int64_t *f, int64_t *cost, int64_t *work)
{
    for (int32_t k = 0; k < n; ++k)
        if (q[k] < 0 || q[k] > Q) return OR_E_DEMAND;
    f[0] = 0;
    int64_t w_extra = 0;
    for (int32_t i = 1; i <= n; ++i) {
        /* positions are 1-based: customer at position k is tour[k-1] */
        int64_t best = INT64_MAX;
        int64_t load = 0;
        int64_t inner = 0; /* sum_{k=p+1}^{i-1} c(s_k, s_{k+1}) */
        int32_t feasible = 0;
        for (int32_t p = i - 1; p >= 0; --p) {
            load += q[p]; /* q_{s_{p+1}} */
            if (load > Q) break;
            if (p < i - 1) inner += DIST(tour[p], tour[p + 1]);
            int64_t route = DIST(0, tour[p]) + inner + DIST(tour[i - 1], 0);
            int64_t cand = f[p] + route;
            if (cand < best) best = cand;
            ++feasible;
        }
        if (feasible == 0) return OR_E_DEMAND;
        w_extra += feasible - 1;
        f[i] = best;
    }
    *cost = f[n];
    *work += w_extra;
    return OR_OK;
}

typedef struct {
    const int32_t *tour;
    int32_t n, N;
    const int32_t *d;
    const int16_t *dem;
    int64_t ld, s_begin, s_end;
    int32_t Q;
    int32_t *cost_out;
    int64_t work;
    int rc;
} or_job;

static void *split_worker(void *arg)
{
    or_job *jb = (or_job *)arg;
    int64_t V = (int64_t)jb->N + 1;
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * ((size_t)jb->n + 1));
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)jb->n);
    if (!f || !q) {
        jb->rc = OR_E_NOMEM;
        free(f);
        free(q);
        return NULL;
    }
    jb->rc = OR_OK;
    for (int64_t s = jb->s_begin; s < jb->s_end; ++s) {
        for (int32_t k = 0; k < jb->n; ++k)
            q[k] = jb->dem[(int64_t)(jb->tour[k] - 1) * jb->ld + s];
        int64_t c = 0;
        int rc = split_one(jb->tour, jb->n, jb->d, V, q, jb->Q, f, &c, &jb->work);
        if (rc != OR_OK) {
            jb->rc = rc;
            break;
        }
        if (c > INT32_MAX) {
            jb->rc = OR_E_INVAL;
            break;
        }
        jb->cost_out[s] = (int32_t)c;
    }
    free(f);
    free(q);
    return NULL;
}

/*
 * Split every scenario s in [0, S) of demand[N][ld] (row c-1 = customer c) along the tour,
 * writing cost_out[s] = f(n). *work_out (optional) receives sum over scenarios and positions
 * of (w_i - 1), the number of pairwise minimisations Eq. (3) needs. nthreads >= 1 threads
 * take contiguous scenario ranges.
 */
int or_split(const int32_t *tour, int32_t n, const int32_t *d, int32_t N, const int16_t *demand,
             int64_t S, int64_t ld, int32_t Q, int32_t *cost_out, int64_t *work_out, int nthreads)
{
    if (!tour || !d || !demand || !cost_out || n < 1 || N < 1 || n > N || S < 1 || ld < S ||
        Q < 1)
        return OR_E_INVAL;
    int rc = check_tour(tour, n, N);
    if (rc != OR_OK) return rc;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > S) nthreads = (int)S;
    or_job jobs[256];
    pthread_t th[256];
    int64_t per = (S + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        or_job *jb = &jobs[t];
        jb->tour = tour; jb->n = n; jb->N = N; jb->d = d; jb->dem = demand; jb->ld = ld;
        jb->Q = Q; jb->cost_out = cost_out; jb->work = 0; jb->rc = OR_OK;
        jb->s_begin = (int64_t)t * per;
        jb->s_end = jb->s_begin + per < S ? jb->s_begin + per : S;
        if (jb->s_begin >= jb->s_end) break;
        if (nthreads == 1) {
            split_worker(jb);
            started = 1;
            break;
        }
        if (pthread_create(&th[t], NULL, split_worker, jb) != 0) return OR_E_NOMEM;
        ++started;
    }
    if (nthreads > 1)
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    int64_t work = 0;
    rc = OR_OK;
    for (int t = 0; t < started; ++t) {
        work += jobs[t].work;
        if (jobs[t].rc != OR_OK && rc == OR_OK) rc = jobs[t].rc;
    }
    if (work_out) *work_out = work;
    return rc;
}

/*
 * Eq. (2) for one scenario: mask_out[i-1] = mask(i), i = 1..n, or -1 when the set is empty
 * (the customer at position i alone exceeds Q). q_pos[k] is the demand at tour position k+1.
 */
int or_mask(const int32_t *q_pos, int32_t n, int32_t Q, int32_t *mask_out)
{
    if (!q_pos || !mask_out || n < 1) return OR_E_INVAL;
    for (int32_t i = 1; i <= n; ++i) {
        int32_t m = -1;
        for (int32_t p = 0; p < i; ++p) {
            int64_t load = 0;
            for (int32_t k = p + 1; k <= i; ++k) load += q_pos[k - 1];
            if (load <= Q) {
                m = p;
                break;
            }
        }
        mask_out[i - 1] = m;
    }
    return OR_OK;
}

/*
 * Eq. (3) for one scenario, given Eq. (2)'s mask: the minimum over p in [mask(i), i-1] with
 * no capacity test, route costs summed term by term. Used to check that Eq. (1) and Eq. (3)
 * agree. Returns f(n) through *cost.
 */
int or_split_masked(const int32_t *tour, int32_t n, const int32_t *d, int32_t N,
                    const int32_t *mask, int64_t *cost)
{
    if (!tour || !d || !mask || !cost || n < 1 || N < 1) return OR_E_INVAL;
    int64_t V = (int64_t)N + 1;
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!f) return OR_E_NOMEM;
    f[0] = 0;
    for (int32_t i = 1; i <= n; ++i) {
        if (mask[i - 1] < 0 || mask[i - 1] > i - 1) {
            free(f);
            return OR_E_DEMAND;
        }
        int64_t best = INT64_MAX;
        for (int32_t p = mask[i - 1]; p <= i - 1; ++p) {
            int64_t route = DIST(0, tour[p]);
            for (int32_t k = p + 1; k <= i - 1; ++k) route += DIST(tour[k - 1], tour[k]);
            route += DIST(tour[i - 1], 0);
            if (f[p] + route < best) best = f[p] + route;
        }
        f[i] = best;
    }
    *cost = f[n];
    free(f);
    return OR_OK;
}

/*
 * Sample-average moments of the scenario costs: exact sum and sum of squares (128-bit,
 * returned as two 64-bit halves), mean = sum / S and the sample variance
 *     var = ((S * sumsq - sum^2) / S) / (S - 1)      (0 when S = 1),
 * where the numerator is exact and converted to double once. Costs must be >= 0.
 */
int or_moments(const int32_t *cost, int64_t S, int64_t *sum_out, uint64_t *sumsq_lo,
               uint64_t *sumsq_hi, double *mean, double *var)
{
    if (!cost || S < 1) return OR_E_INVAL;
    unsigned __int128 sum = 0, sumsq = 0;
    for (int64_t s = 0; s < S; ++s) {
        if (cost[s] < 0) return OR_E_INVAL;
        uint64_t c = (uint64_t)cost[s];
        sum += c;
        sumsq += (unsigned __int128)(c * c);
    }
    if (sum_out) *sum_out = (int64_t)sum;
    if (sumsq_lo) *sumsq_lo = (uint64_t)sumsq;
    if (sumsq_hi) *sumsq_hi = (uint64_t)(sumsq >> 64);
    if (mean) *mean = (double)(int64_t)sum / (double)S;
    if (var) {
        if (S == 1) {
            *var = 0.0;
        } else {
            unsigned __int128 num = (unsigned __int128)S * sumsq - sum * sum;
            *var = ((double)num / (double)S) / (double)(S - 1);
        }
    }
    return OR_OK;
}

/*
 * Strong CPU baseline (a timing reference, not a correctness reference): the linear-time
 * Split for an unlimited fleet (Vidal, "Technical note: Split algorithm in O(n) for the
 * capacitated vehicle routing problem", Computers & Operations Research 69, 2016), one
 * scenario at a time, threads over contiguous scenario ranges.
 *
 * With A[k] = sum of the tour arcs from position 1 to position k (A[1] = 0), the route of
 * positions p+1..i costs d[0][s_{p+1}] + A[i] - A[p+1] + d[s_i][0], so
 *     f(i) = A[i] + d[s_i][0] + min over the feasible p of  key(p),
 *     key(p) = f(p) + d[0][s_{p+1}] - A[p+1].
 * The feasible p of state i form the window [start(i), i-1] of Eq. (2), whose start never
 * decreases with i (demands are >= 0). A deque of predecessors kept increasing in key gives
 * each window minimum at its front: a predecessor leaves at the front once the window start
 * passes it, and at the back once a later one has a key no larger. Each p enters and leaves
 * once: O(n) per scenario. The tests check it against or_split on every scenario.
 */
typedef struct {
    int32_t n;
    const int32_t *tour;
    const int64_t *A, *out0, *back0;
    const int16_t *dem;
    int64_t ld, s_begin, s_end;
    int32_t Q;
    int32_t *cost_out;
    int rc;
} or_deque_job;

/* One scenario: q[k] is the demand at tour position k+1; P, key and dq are scratch of n+1. */
static int deque_one(int32_t n, const int64_t *A, const int64_t *out0, const int64_t *back0,
                     const int16_t *q, int32_t Q, int64_t *P, int64_t *key, int32_t *dq,
                     int64_t *cost)
{
    P[0] = 0;
    for (int32_t k = 1; k <= n; ++k) {
        if (q[k - 1] < 0 || q[k - 1] > Q) return OR_E_DEMAND;
        P[k] = P[k - 1] + q[k - 1];
    }
    int32_t head = 0, tail = 0, start = 0;
    int64_t f = 0;
    key[0] = out0[0] - A[1]; /* f(0) = 0 */
    dq[tail++] = 0;
    for (int32_t i = 1; i <= n; ++i) {
        while (P[i] - P[start] > Q) ++start;
        while (head < tail && dq[head] < start) ++head;
        if (head == tail) return OR_E_DEMAND; /* not reached once q_i <= Q: p = i-1 is feasible */
        f = key[dq[head]] + A[i] + back0[i];
        if (i < n) {
            key[i] = f + out0[i] - A[i + 1];
            while (head < tail && key[dq[tail - 1]] >= key[i]) --tail;
            dq[tail++] = i;
        }
    }
    *cost = f;
    return OR_OK;
}

#define OR_DEQUE_BLOCK 32 /* scenarios whose demand rows are copied out together */

static void *deque_worker(void *arg)
{
    or_deque_job *jb = (or_deque_job *)arg;
    const int32_t n = jb->n;
    int64_t *P = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *dq = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    /* the block's demands, scenario-major: qb[b * n + k] = demand of scenario s0 + b at tour
       position k + 1 (one pass over each demand row, then contiguous reads per scenario) */
    int16_t *qb = (int16_t *)malloc(sizeof(int16_t) * (size_t)n * OR_DEQUE_BLOCK);
    jb->rc = (P && key && dq && qb) ? OR_OK : OR_E_NOMEM;
    for (int64_t s0 = jb->s_begin; s0 < jb->s_end && jb->rc == OR_OK; s0 += OR_DEQUE_BLOCK) {
        const int nb = (int)(jb->s_end - s0 < OR_DEQUE_BLOCK ? jb->s_end - s0 : OR_DEQUE_BLOCK);
        for (int32_t k = 0; k < n; ++k) {
            const int16_t *row = jb->dem + (int64_t)(jb->tour[k] - 1) * jb->ld + s0;
            for (int b = 0; b < nb; ++b) qb[(size_t)b * n + k] = row[b];
        }
        for (int b = 0; b < nb; ++b) {
            int64_t c = 0;
            int rc = deque_one(n, jb->A, jb->out0, jb->back0, qb + (size_t)b * n, jb->Q, P, key,
                               dq, &c);
            if (rc == OR_OK && c > INT32_MAX) rc = OR_E_INVAL;
            if (rc != OR_OK) {
                jb->rc = rc;
                break;
            }
            jb->cost_out[s0 + b] = (int32_t)c;
        }
    }
    free(P);
    free(key);
    free(dq);
    free(qb);
    return NULL;
}

/* The same contract as or_split (without the work count), computed by the linear Split. */
int or_split_deque(const int32_t *tour, int32_t n, const int32_t *d, int32_t N,
                   const int16_t *demand, int64_t S, int64_t ld, int32_t Q, int32_t *cost_out,
                   int nthreads)
{
    if (!tour || !d || !demand || !cost_out || n < 1 || N < 1 || n > N || S < 1 || ld < S ||
        Q < 1)
        return OR_E_INVAL;
    int rc = check_tour(tour, n, N);
    if (rc != OR_OK) return rc;
    const int64_t V = (int64_t)N + 1;
    /* tour arrays shared by every scenario: A[1..n], out0[0..n-1], back0[1..n] */
    int64_t *A = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *out0 = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *back0 = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!A || !out0 || !back0) {
        free(A);
        free(out0);
        free(back0);
        return OR_E_NOMEM;
    }
    A[0] = 0;
    A[1] = 0;
    for (int32_t k = 2; k <= n; ++k) A[k] = A[k - 1] + DIST(tour[k - 2], tour[k - 1]);
    for (int32_t p = 0; p < n; ++p) out0[p] = DIST(0, tour[p]);
    back0[0] = 0;
    for (int32_t i = 1; i <= n; ++i) back0[i] = DIST(tour[i - 1], 0);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > S) nthreads = (int)S;
    or_deque_job jobs[256];
    pthread_t th[256];
    int64_t per = (S + nthreads - 1) / nthreads;
    int started = 0;
    rc = OR_OK;
    for (int t = 0; t < nthreads; ++t) {
        or_deque_job *jb = &jobs[t];
        jb->n = n; jb->tour = tour; jb->A = A; jb->out0 = out0; jb->back0 = back0;
        jb->dem = demand; jb->ld = ld; jb->Q = Q; jb->cost_out = cost_out; jb->rc = OR_OK;
        jb->s_begin = (int64_t)t * per;
        jb->s_end = jb->s_begin + per < S ? jb->s_begin + per : S;
        if (jb->s_begin >= jb->s_end) break;
        if (nthreads == 1) {
            deque_worker(jb);
            started = 1;
            break;
        }
        if (pthread_create(&th[t], NULL, deque_worker, jb) != 0) {
            rc = OR_E_NOMEM;
            break;
        }
        ++started;
    }
    if (nthreads > 1)
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < started; ++t)
        if (jobs[t].rc != OR_OK && rc == OR_OK) rc = jobs[t].rc;
    free(A);
    free(out0);
    free(back0);
    return rc;
}
