/*
 * Seeded synthetic inputs for the scenario-batched Split: instance coordinates, giant
 * tours and demand scenarios.
 *
 * This module is shared by the GPU library's tests/bench and by the CPU oracle's tests.
 * It holds none of the Split arithmetic: it only draws random numbers and shapes them into
 * the input arrays (coordinates, permutations, int16 demand matrices).
 *
 * Random numbers come from the counter-based generator Philox4x32-10, written from its
 * published definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): a 4x32-bit counter, a 2x32-bit key, ten rounds of two 32x32->64
 * multiplications with the multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by the
 * Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds. Every drawn value is a pure
 * function of (seed, stream, indices), so the arrays do not depend on the thread count.
 *
 * Demand layout: int16 dem[c-1][ld] for customer c = 1..N, scenario index fastest.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    SG_STREAM_COORDS = 1,
    SG_STREAM_TOUR = 2,
    SG_STREAM_UNIFORM = 3,
    SG_STREAM_LAMBDA = 4,
    SG_STREAM_POISSON = 5,
    SG_STREAM_COPULA = 6,
    SG_STREAM_PERTURB = 8,
};

void sg_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One Philox block for (seed, stream, a, b): counter = (a_lo, a_hi, b, stream). */
static void draw4(uint64_t seed, uint32_t stream, uint64_t a, uint32_t b, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)a, (uint32_t)(a >> 32), b, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    sg_philox4x32_10(ctr, key, out);
}

/* Uniform on (0, 1]: never 0, so log() is finite. */
static double u01_open0(uint32_t x) { return ((double)x + 1.0) * (1.0 / 4294967296.0); }
/* Uniform on [0, 1). */
static double u01(uint32_t x) { return (double)x * (1.0 / 4294967296.0); }

/* Box-Muller: one standard normal from two 32-bit words. */
static double normal_from(uint32_t w0, uint32_t w1)
{
    const double two_pi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(u01_open0(w0))) * cos(two_pi * u01(w1));
}

/* Integer coordinates uniform on {0..grid-1}^2 for nodes 0..N (node 0 is the depot). */
int sg_coords(uint64_t seed, int32_t N, int32_t grid, int32_t *xy)
{
    if (N < 1 || grid < 1 || !xy) return -1;
    for (int32_t v = 0; v <= N; ++v) {
        uint32_t r[4];
        draw4(seed, SG_STREAM_COORDS, (uint64_t)v, 0, r);
        xy[2 * v + 0] = (int32_t)(((uint64_t)r[0] * (uint64_t)grid) >> 32);
        xy[2 * v + 1] = (int32_t)(((uint64_t)r[1] * (uint64_t)grid) >> 32);
    }
    return 0;
}

/*
 * Seeded uniformly random permutation of the customers 1..N (Fisher-Yates driven by
 * Philox); the first n entries are returned, so n < N gives a random subset tour.
 * `variant` selects an independent permutation for the same seed.
 */
int sg_tour(uint64_t seed, uint32_t variant, int32_t N, int32_t n, int32_t *tour)
{
    if (N < 1 || n < 1 || n > N || !tour) return -1;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!perm) return -2;
    for (int32_t k = 0; k < N; ++k) perm[k] = k + 1;
    for (int32_t k = N - 1; k > 0; --k) {
        uint32_t r[4];
        draw4(seed, SG_STREAM_TOUR, (uint64_t)k, variant, r);
        int32_t j = (int32_t)(((uint64_t)r[0] * (uint64_t)(k + 1)) >> 32);
        int32_t t = perm[k];
        perm[k] = perm[j];
        perm[j] = t;
    }
    memcpy(tour, perm, sizeof(int32_t) * (size_t)n);
    free(perm);
    return 0;
}

/* ---- demand matrices, threaded over contiguous scenario ranges ---- */

typedef struct {
    int kind; /* 0 uniform, 1 poisson, 2 copula */
    uint64_t seed;
    int32_t N;
    int64_t s_begin, s_end, ld;
    int16_t *dem;
    /* uniform */
    int32_t lo, hi;
    /* poisson */
    const double *lam;
    /* copula */
    double rho, mu_ln, sigma_ln;
    int32_t Q;
} sg_job;

static int16_t clip_q(long long v, int32_t Q)
{
    if (v < 0) v = 0;
    if (v > Q) v = Q;
    return (int16_t)v;
}

static void *sg_worker(void *arg)
{
    sg_job *jb = (sg_job *)arg;
    const int64_t CH = 2048;
    double *z = NULL;
    if (jb->kind == 2) {
        z = (double *)malloc(sizeof(double) * (size_t)CH);
        if (!z) return (void *)1;
    }
    for (int64_t s0 = jb->s_begin; s0 < jb->s_end; s0 += CH) {
        int64_t s1 = s0 + CH < jb->s_end ? s0 + CH : jb->s_end;
        for (int32_t c = 1; c <= jb->N; ++c) {
            int16_t *row = jb->dem + (int64_t)(c - 1) * jb->ld;
            for (int64_t s = s0; s < s1; ++s) {
                uint32_t r[4];
                if (jb->kind == 0) {
                    draw4(jb->seed, SG_STREAM_UNIFORM, (uint64_t)s, (uint32_t)c, r);
                    uint32_t span = (uint32_t)(jb->hi - jb->lo + 1);
                    row[s] = (int16_t)(jb->lo + (int32_t)(((uint64_t)r[0] * span) >> 32));
                } else if (jb->kind == 1) {
                    draw4(jb->seed, SG_STREAM_POISSON, (uint64_t)s, (uint32_t)c, r);
                    double u = u01(r[0]);
                    double lam = jb->lam[c - 1];
                    double p = exp(-lam), F = p;
                    int32_t k = 0;
                    while (u > F && k < jb->Q) {
                        ++k;
                        p *= lam / (double)k;
                        F += p;
                    }
                    row[s] = clip_q(k, jb->Q);
                } else {
                    draw4(jb->seed, SG_STREAM_COPULA, (uint64_t)s, (uint32_t)c, r);
                    double eps = normal_from(r[0], r[1]);
                    double *zz = &z[s - s0];
                    if (c == 1)
                        *zz = eps;
                    else
                        *zz = jb->rho * *zz + sqrt(1.0 - jb->rho * jb->rho) * eps;
                    double q = exp(jb->mu_ln + jb->sigma_ln * *zz);
                    row[s] = clip_q(llround(q), jb->Q);
                }
            }
        }
    }
    free(z);
    return NULL;
}

static int run_jobs(sg_job proto, int64_t S, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > S) nthreads = (int)S;
    pthread_t th[256];
    sg_job jobs[256];
    int64_t per = (S + nthreads - 1) / nthreads;
    int started = 0, rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = proto;
        jobs[t].s_begin = (int64_t)t * per;
        jobs[t].s_end = jobs[t].s_begin + per < S ? jobs[t].s_begin + per : S;
        if (jobs[t].s_begin >= jobs[t].s_end) break;
        if (pthread_create(&th[t], NULL, sg_worker, &jobs[t]) != 0) {
            rc = -3;
            break;
        }
        ++started;
    }
    for (int t = 0; t < started; ++t) {
        void *ret = NULL;
        pthread_join(th[t], &ret);
        if (ret) rc = -2;
    }
    return rc;
}

/* q ~ U{lo..hi} iid. */
int sg_demand_uniform(uint64_t seed, int32_t N, int64_t S, int64_t ld, int32_t lo, int32_t hi,
                      int16_t *dem, int nthreads)
{
    if (N < 1 || S < 1 || ld < S || lo > hi || lo < -32768 || hi > 32767 || !dem) return -1;
    sg_job jb;
    memset(&jb, 0, sizeof jb);
    jb.kind = 0; jb.seed = seed; jb.N = N; jb.ld = ld; jb.dem = dem; jb.lo = lo; jb.hi = hi;
    return run_jobs(jb, S, nthreads);
}

/*
 * q ~ Poisson(lambda_c) iid by CDF inversion, clipped to [0, Q]; lambda_c ~ U[lam_lo, lam_hi]
 * (continuous) fixed per customer. lam_out (optional, N doubles) receives the lambdas.
 */
int sg_demand_poisson(uint64_t seed, int32_t N, int64_t S, int64_t ld, double lam_lo,
                      double lam_hi, int32_t Q, int16_t *dem, double *lam_out, int nthreads)
{
    if (N < 1 || S < 1 || ld < S || Q < 1 || Q > 32767 || !(lam_lo > 0) || lam_hi < lam_lo ||
        lam_hi > 700.0 || !dem)
        return -1;
    double *lam = (double *)malloc(sizeof(double) * (size_t)N);
    if (!lam) return -2;
    for (int32_t c = 1; c <= N; ++c) {
        uint32_t r[4];
        draw4(seed, SG_STREAM_LAMBDA, (uint64_t)c, 0, r);
        lam[c - 1] = lam_lo + (lam_hi - lam_lo) * u01(r[0]);
    }
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * (size_t)N);
    sg_job jb;
    memset(&jb, 0, sizeof jb);
    jb.kind = 1; jb.seed = seed; jb.N = N; jb.ld = ld; jb.dem = dem; jb.lam = lam; jb.Q = Q;
    int rc = run_jobs(jb, S, nthreads);
    free(lam);
    return rc;
}

/*
 * Gaussian-copula demands: Z_1 = e_1, Z_c = rho Z_{c-1} + sqrt(1 - rho^2) e_c along the
 * customer id (e_c iid standard normal), lognormal marginal with the given mean and
 * coefficient of variation, rounded to the nearest integer and clipped to [0, Q].
 */
int sg_demand_copula(uint64_t seed, int32_t N, int64_t S, int64_t ld, double rho, double mean,
                     double cv, int32_t Q, int16_t *dem, int nthreads)
{
    if (N < 1 || S < 1 || ld < S || Q < 1 || Q > 32767 || !(rho > -1.0 && rho < 1.0) ||
        !(mean > 0) || !(cv > 0) || !dem)
        return -1;
    double s2 = log(1.0 + cv * cv);
    sg_job jb;
    memset(&jb, 0, sizeof jb);
    jb.kind = 2; jb.seed = seed; jb.N = N; jb.ld = ld; jb.dem = dem; jb.Q = Q;
    jb.rho = rho; jb.sigma_ln = sqrt(s2); jb.mu_ln = log(mean) - 0.5 * s2;
    return run_jobs(jb, S, nthreads);
}

/* ---- candidate tours for the surrogate's training and screening ---- */

static double edist(const int32_t *xy, int32_t u, int32_t v)
{
    const double dx = (double)xy[2 * u] - (double)xy[2 * v];
    const double dy = (double)xy[2 * u + 1] - (double)xy[2 * v + 1];
    return sqrt(dx * dx + dy * dy);
}

/*
 * A short giant tour over customers 1..N: nearest neighbour from the depot, then 2-opt
 * (reverse tour[i..j] when it shortens the closed depot-tour-depot cycle; first improvement)
 * until a sweep improves nothing or max_passes sweeps. Straight-line double distances: this is
 * only a good starting point for perturbed candidates, not any cost the Split computes.
 */
int sg_two_opt_tour(const int32_t *xy, int32_t N, int32_t max_passes, int32_t *tour)
{
    if (!xy || !tour || N < 1) return -1;
    unsigned char *used = (unsigned char *)calloc((size_t)N + 1, 1);
    if (!used) return -2;
    int32_t cur = 0;
    for (int32_t k = 0; k < N; ++k) {
        int32_t best = -1;
        double bd = 0.0;
        for (int32_t c = 1; c <= N; ++c) {
            if (used[c]) continue;
            const double dd = edist(xy, cur, c);
            if (best < 0 || dd < bd) {
                best = c;
                bd = dd;
            }
        }
        used[best] = 1;
        tour[k] = best;
        cur = best;
    }
    free(used);
    for (int32_t pass = 0; pass < max_passes; ++pass) {
        int improved = 0;
        for (int32_t i = 0; i < N - 1; ++i) {
            const int32_t a = i > 0 ? tour[i - 1] : 0;
            for (int32_t j = i + 1; j < N; ++j) {
                const int32_t b = j + 1 < N ? tour[j + 1] : 0;
                const double delta = edist(xy, a, tour[j]) + edist(xy, tour[i], b) -
                                     edist(xy, a, tour[i]) - edist(xy, tour[j], b);
                if (delta < -1e-9) {
                    for (int32_t l = i, r = j; l < r; ++l, --r) {
                        const int32_t t = tour[l];
                        tour[l] = tour[r];
                        tour[r] = t;
                    }
                    improved = 1;
                }
            }
        }
        if (!improved) break;
    }
    return 0;
}

typedef struct {
    uint64_t seed;
    const int32_t *base;
    int32_t n, rmin, rmax;
    int64_t c_begin, c_end;
    int32_t *out;
} sg_pjob;

static void *sg_perturb_worker(void *arg)
{
    const sg_pjob *j = (const sg_pjob *)arg;
    for (int64_t c = j->c_begin; c < j->c_end; ++c) {
        int32_t *t = j->out + c * j->n;
        memcpy(t, j->base, sizeof(int32_t) * (size_t)j->n);
        uint32_t r[4];
        draw4(j->seed, SG_STREAM_PERTURB, (uint64_t)c, 0xFFFFFFFFu, r);
        const int32_t span = j->rmax - j->rmin + 1;
        const int32_t moves = j->rmin + (int32_t)(((uint64_t)r[0] * (uint64_t)span) >> 32);
        for (int32_t k = 0; k < moves; ++k) {
            draw4(j->seed, SG_STREAM_PERTURB, (uint64_t)c, (uint32_t)k, r);
            int32_t a = (int32_t)(((uint64_t)r[0] * (uint64_t)j->n) >> 32);
            int32_t b = (int32_t)(((uint64_t)r[1] * (uint64_t)j->n) >> 32);
            if (a > b) {
                const int32_t x = a;
                a = b;
                b = x;
            }
            for (; a < b; ++a, --b) {
                const int32_t x = t[a];
                t[a] = t[b];
                t[b] = x;
            }
        }
    }
    return NULL;
}

/*
 * count candidates [count][n]: the base tour with m random segment reversals each, m uniform
 * on {rmin..rmax}; reversal k of candidate c reverses positions [min(a,b), max(a,b)] with a, b
 * uniform on {0..n-1} from Philox (seed, stream 8, counter (c, k)). Threads over candidates.
 */
int sg_perturb(uint64_t seed, const int32_t *base, int32_t n, int64_t count, int32_t rmin,
               int32_t rmax, int32_t *out, int nthreads)
{
    if (!base || !out || n < 1 || count < 0 || rmin < 0 || rmax < rmin) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    sg_pjob jobs[64];
    int started = 0;
    for (int k = 0; k < nthreads; ++k) {
        jobs[k].seed = seed;
        jobs[k].base = base;
        jobs[k].n = n;
        jobs[k].rmin = rmin;
        jobs[k].rmax = rmax;
        jobs[k].c_begin = count * k / nthreads;
        jobs[k].c_end = count * (k + 1) / nthreads;
        jobs[k].out = out;
        /* a thread that cannot start runs its share here */
        if (pthread_create(&th[started], NULL, sg_perturb_worker, &jobs[k]) == 0)
            ++started;
        else
            sg_perturb_worker(&jobs[k]);
    }
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    return 0;
}
