// Drives every C-ABI entry point of the library (split.h, split_nn.h, split_search.h) on small
// seeded inputs, for a build whose host code runs under AddressSanitizer and
// UndefinedBehaviorSanitizer (the device code is the library's own). A sanitizer report aborts
// the process; any unexpected status or any disagreement between the evaluation paths makes it
// exit with status 1 after printing what differed. Every path computes exactly Section 3's
// Eqs. (1)-(3), so the kernel forms, block lengths, batch, graph and allocation-free entry
// points must agree bit for bit.
//
// Usage: host_sanitize_driver <scratch directory for a checkpoint file>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../include/split.h"
#include "../include/split_nn.h"
#include "../include/split_search.h"

namespace {

int g_fail = 0;

#define EXPECT(cond, ...)                                                 \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);          \
            fprintf(stderr, __VA_ARGS__);                                 \
            fprintf(stderr, "\n");                                        \
            ++g_fail;                                                     \
        }                                                                 \
    } while (0)

#define HIP_OK(call)                                                             \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            fprintf(stderr, "HIP %s at %s:%d\n", hipGetErrorString(e_), __FILE__, \
                    __LINE__);                                                   \
            return 1;                                                            \
        }                                                                        \
    } while (0)

// splitmix64: the driver's own seeded inputs
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int uniform(int lo, int hi) { return lo + (int)(next() % (uint64_t)(hi - lo + 1)); }
};

std::vector<int32_t> permutation(Rng &r, int N, int n)
{
    std::vector<int32_t> p(N);
    for (int i = 0; i < N; ++i) p[i] = i + 1;
    for (int i = N - 1; i > 0; --i) std::swap(p[i], p[r.uniform(0, i)]);
    p.resize(n);
    return p;
}

std::vector<int32_t> to_host(const int32_t *d, size_t count)
{
    std::vector<int32_t> h(count);
    if (hipMemcpy(h.data(), d, count * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        h.assign(count, -7);
    return h;
}

bool same_stats(const split_stats &a, const split_stats &b)
{
    return a.sum == b.sum && a.sumsq_lo == b.sumsq_lo && a.sumsq_hi == b.sumsq_hi &&
           a.mean == b.mean && a.var == b.var;
}

}  // namespace

int main(int argc, char **argv)
{
    const std::string scratch = argc > 1 ? argv[1] : "/tmp";
    const int N = 300, S = 1500, Q = 200;
    Rng rng{12345};

    // instance, demands (two laws: windows of about 10 and about 25 customers)
    std::vector<int32_t> xy(2 * (N + 1));
    for (auto &v : xy) v = rng.uniform(0, 999);
    std::vector<int16_t> dem((size_t)N * S);
    for (int c = 0; c < N; ++c)
        for (int s = 0; s < S; ++s)
            dem[(size_t)c * S + s] = (int16_t)(s < S / 2 ? rng.uniform(5, 35) : rng.uniform(0, 16));
    int16_t *d_dem = nullptr;
    int32_t *d_cost = nullptr, *d_cost2 = nullptr;
    const int Tmax = 6;
    HIP_OK(hipMalloc(&d_dem, dem.size() * sizeof(int16_t)));
    HIP_OK(hipMemcpy(d_dem, dem.data(), dem.size() * sizeof(int16_t), hipMemcpyHostToDevice));
    HIP_OK(hipMalloc(&d_cost, (size_t)Tmax * S * sizeof(int32_t)));
    HIP_OK(hipMalloc(&d_cost2, (size_t)Tmax * S * sizeof(int32_t)));

    split_ctx *ctx = nullptr;
    EXPECT(split_ctx_create(0, &ctx) == SPLIT_OK && ctx, "ctx_create");
    if (!ctx) return 1;
    EXPECT(split_instance_set_coords(ctx, N, xy.data()) == SPLIT_OK, "set_coords: %s",
           split_last_error(ctx));

    // one tour under every form and block length, blocking and enqueued
    const std::vector<int32_t> tour = permutation(rng, N, 240);
    const int n = (int)tour.size();
    split_stats ref_st{};
    std::vector<int32_t> ref;
    const split_tuning choices[] = {{SPLIT_FORM_LANE, 0, 0, 0, 16}, {SPLIT_FORM_LANE, 0, 0, 0, 8},
                                    {SPLIT_FORM_LANE, 4, 1, 0, 8},  {SPLIT_FORM_WAVE, 0, 0, 0, 0},
                                    {SPLIT_FORM_WAVE, 0, 0, 512, 0}, {SPLIT_FORM_MASK, 0, 0, 0, 0},
                                    {SPLIT_FORM_AUTO, 0, 0, 0, 0}};
    for (const split_tuning &tu : choices) {
        EXPECT(split_tuning_set(ctx, &tu) == SPLIT_OK, "tuning_set");
        split_tuning back{};
        EXPECT(split_tuning_get(ctx, &back) == SPLIT_OK && memcmp(&back, &tu, sizeof tu) == 0,
               "tuning_get");
        split_stats st{};
        EXPECT(split_eval(ctx, tour.data(), n, d_dem, S, S, Q, d_cost, &st, nullptr) == SPLIT_OK,
               "eval form %d block %d: %s", tu.form, tu.lane_block, split_last_error(ctx));
        const std::vector<int32_t> got = to_host(d_cost, S);
        if (ref.empty()) {
            ref = got;
            ref_st = st;
        } else {
            EXPECT(got == ref, "form %d block %d differs", tu.form, tu.lane_block);
            EXPECT(same_stats(st, ref_st), "form %d block %d statistics differ", tu.form,
                   tu.lane_block);
        }
        // enqueued call, statistics collected later
        EXPECT(split_eval(ctx, tour.data(), n, d_dem, S, S, Q, d_cost2, nullptr, nullptr) ==
                   SPLIT_OK, "async eval");
        split_stats st2{};
        EXPECT(split_stats_get(ctx, &st2) == SPLIT_OK && same_stats(st2, ref_st), "stats_get");
    }
    EXPECT(to_host(d_cost2, S) == ref, "async costs differ");

    // allocation-free entry point, twice (the second with fewer scenarios)
    const split_tuning lane16 = {SPLIT_FORM_LANE, 0, 0, 0, 0};
    EXPECT(split_tuning_set(ctx, &lane16) == SPLIT_OK, "tuning_set");
    for (int rep = 0; rep < 2; ++rep) {
        const int Sx = rep == 0 ? S : S / 3;
        split_stats st{};
        EXPECT(split_eval_noalloc(ctx, tour.data(), n, d_dem, Sx, S, Q, d_cost2, &st, nullptr) ==
                   SPLIT_OK, "noalloc: %s", split_last_error(ctx));
        const std::vector<int32_t> got = to_host(d_cost2, Sx);
        EXPECT(std::equal(got.begin(), got.end(), ref.begin()), "noalloc rep %d differs", rep);
    }

    // batch of uneven tours, timing on
    std::vector<int32_t> flat;
    std::vector<int64_t> ptr{0};
    std::vector<std::vector<int32_t>> tours;
    for (int t = 0; t < Tmax; ++t) {
        tours.push_back(t == 0 ? tour : permutation(rng, N, rng.uniform(1, N)));
        flat.insert(flat.end(), tours.back().begin(), tours.back().end());
        ptr.push_back((int64_t)flat.size());
    }
    EXPECT(split_timing_enable(ctx, 1) == SPLIT_OK, "timing_enable");
    EXPECT(split_timing_reset(ctx) == SPLIT_OK, "timing_reset");
    std::vector<split_stats> bst(Tmax);
    std::vector<int32_t> bstatus(Tmax, -9);
    EXPECT(split_eval_batch(ctx, flat.data(), ptr.data(), Tmax, d_dem, S, S, Q, d_cost, S,
                            bst.data(), bstatus.data(), nullptr) == SPLIT_OK,
           "eval_batch: %s", split_last_error(ctx));
    const std::vector<int32_t> batch = to_host(d_cost, (size_t)Tmax * S);
    EXPECT(std::equal(ref.begin(), ref.end(), batch.begin()), "batch row 0 differs");
    for (int t = 0; t < Tmax; ++t) {
        EXPECT(bstatus[t] == SPLIT_OK, "batch status %d", t);
        split_stats st{};
        EXPECT(split_eval(ctx, tours[t].data(), (int)tours[t].size(), d_dem, S, S, Q, d_cost2, &st,
                          nullptr) == SPLIT_OK, "eval tour %d", t);
        const std::vector<int32_t> one = to_host(d_cost2, S);
        EXPECT(std::equal(one.begin(), one.end(), batch.begin() + (size_t)t * S),
               "batch row %d differs", t);
        EXPECT(same_stats(st, bst[t]), "batch statistics %d differ", t);
    }
    double ms = 0.0;
    int64_t launches = 0, count = 0;
    const char *kname = nullptr;
    EXPECT(split_timing_get(ctx, &ms, &launches, &kname) == SPLIT_OK && launches > 0 && kname,
           "timing_get");
    EXPECT(split_timing_samples(ctx, nullptr, 0, &count) == SPLIT_OK && count == launches,
           "timing_samples count");
    std::vector<float> samples((size_t)count);
    EXPECT(split_timing_samples(ctx, samples.data(), count, &count) == SPLIT_OK,
           "timing_samples");
    EXPECT(split_timing_enable(ctx, 0) == SPLIT_OK, "timing off");
    std::vector<split_stats> bst2(Tmax);
    EXPECT(split_batch_stats_get(ctx, bst2.data(), bstatus.data()) == SPLIT_OK, "batch_stats_get");

    // autotuner on the batch; the installed choice keeps the costs
    split_tuning best{};
    double best_ms = 0.0;
    EXPECT(split_autotune(ctx, flat.data(), ptr.data(), Tmax, d_dem, S, S, Q, d_cost2, S, 2,
                          nullptr, &best, &best_ms) == SPLIT_OK, "autotune: %s",
           split_last_error(ctx));
    EXPECT(to_host(d_cost2, (size_t)Tmax * S) == batch, "autotuned costs differ");

    // captured graph: two launches with different batches, statistics, destroy
    split_graph *g = nullptr;
    EXPECT(split_graph_create(ctx, Tmax, (int64_t)Tmax * N, d_dem, S, S, Q, d_cost2, S, &g) ==
               SPLIT_OK && g, "graph_create: %s", split_last_error(ctx));
    if (g) {
        for (int rep = 0; rep < 2; ++rep) {
            const int T = rep == 0 ? Tmax : 2;
            EXPECT(split_graph_launch(g, flat.data(), ptr.data(), T, nullptr) == SPLIT_OK,
                   "graph_launch");
            std::vector<split_stats> gst(T);
            std::vector<int32_t> gstatus(T, -9);
            EXPECT(split_graph_stats(g, gst.data(), gstatus.data()) == SPLIT_OK, "graph_stats");
            const std::vector<int32_t> got = to_host(d_cost2, (size_t)T * S);
            EXPECT(std::equal(got.begin(), got.end(), batch.begin()), "graph rep %d differs", rep);
            for (int t = 0; t < T; ++t)
                EXPECT(same_stats(gst[t], bst[t]) && gstatus[t] == SPLIT_OK, "graph stats %d", t);
        }
        // over capacity
        std::vector<int64_t> big{0};
        for (int t = 0; t <= Tmax; ++t) big.push_back(big.back() + 1);
        EXPECT(split_graph_launch(g, flat.data(), big.data(), Tmax + 1, nullptr) == SPLIT_E_INVAL,
               "graph over capacity");
        split_graph_destroy(g);
    }
    split_graph_destroy(nullptr);

    // error paths
    EXPECT(split_eval(nullptr, tour.data(), n, d_dem, S, S, Q, d_cost, nullptr, nullptr) ==
               SPLIT_E_INVAL, "NULL ctx");
    EXPECT(split_eval(ctx, tour.data(), n, d_dem, S, S, 0, d_cost, nullptr, nullptr) ==
               SPLIT_E_INVAL, "Q = 0");
    EXPECT(split_eval(ctx, tour.data(), n, d_dem, S, S - 1, Q, d_cost, nullptr, nullptr) ==
               SPLIT_E_INVAL, "ld < S");
    EXPECT(split_eval(ctx, tour.data(), N + 1, d_dem, S, S, Q, d_cost, nullptr, nullptr) ==
               SPLIT_E_INVAL, "n > N");
    std::vector<int32_t> rep_tour = tour;
    rep_tour[5] = rep_tour[6];
    EXPECT(split_eval(ctx, rep_tour.data(), n, d_dem, S, S, Q, d_cost, nullptr, nullptr) ==
               SPLIT_E_TOUR, "repeated id");
    rep_tour[5] = N + 1;
    EXPECT(split_eval(ctx, rep_tour.data(), n, d_dem, S, S, Q, d_cost, nullptr, nullptr) ==
               SPLIT_E_TOUR, "id out of range");
    split_stats st{};
    EXPECT(split_eval(ctx, tour.data(), n, d_dem, S, S, 30, d_cost, &st, nullptr) ==
               SPLIT_E_DEMAND, "q > Q");
    const split_tuning bad_block = {SPLIT_FORM_LANE, 0, 0, 0, 4};
    EXPECT(split_tuning_set(ctx, &bad_block) == SPLIT_E_INVAL, "lane_block 4");
    const split_tuning mask = {SPLIT_FORM_MASK, 0, 0, 0, 0};
    EXPECT(split_tuning_set(ctx, &mask) == SPLIT_OK, "mask form");
    EXPECT(split_eval_noalloc(ctx, tour.data(), n, d_dem, S, S, Q, d_cost, nullptr, nullptr) ==
               SPLIT_E_INVAL, "noalloc under the mask form");
    EXPECT(split_tuning_set(ctx, &lane16) == SPLIT_OK, "tuning_set");
    EXPECT(split_autotune(ctx, flat.data(), ptr.data(), Tmax, d_dem, S, S, Q, d_cost2, S, 0,
                          nullptr, nullptr, nullptr) == SPLIT_E_INVAL, "autotune reps 0");
    std::vector<int32_t> dist((size_t)(N + 1) * (N + 1), 3);
    dist[7] = -1;
    EXPECT(split_instance_set_dist(ctx, N, dist.data()) == SPLIT_E_INVAL, "negative distance");
    EXPECT(strlen(split_last_error(ctx)) > 0, "last_error");
    dist[7] = 3;
    for (int i = 0; i <= N; ++i) dist[(size_t)i * (N + 1) + i] = 0;
    EXPECT(split_instance_set_dist(ctx, N, dist.data()) == SPLIT_OK, "set_dist");
    EXPECT(split_eval(ctx, tour.data(), n, d_dem, S, S, Q, d_cost, &st, nullptr) == SPLIT_OK,
           "eval on a matrix");
    EXPECT(split_instance_set_coords(ctx, N, xy.data()) == SPLIT_OK, "set_coords again");

    // surrogate: create, features, predict, gradient, train, checkpoint, shortlist, screen
    split_nn *nn = nullptr;
    EXPECT(split_nn_create(ctx, 7, 1000.0, &nn) == SPLIT_OK && nn, "nn_create: %s",
           split_last_error(ctx));
    if (nn) {
        const int T = 8, nt = 120;
        std::vector<int32_t> cand;
        for (int t = 0; t < T; ++t) {
            const std::vector<int32_t> p = permutation(rng, N, nt);
            cand.insert(cand.end(), p.begin(), p.end());
        }
        int32_t *d_tours = nullptr, *d_idx = nullptr;
        float *d_pred = nullptr, *d_lab = nullptr;
        HIP_OK(hipMalloc(&d_tours, cand.size() * sizeof(int32_t)));
        HIP_OK(hipMemcpy(d_tours, cand.data(), cand.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
        HIP_OK(hipMalloc(&d_pred, T * sizeof(float)));
        HIP_OK(hipMalloc(&d_lab, T * sizeof(float)));
        HIP_OK(hipMalloc(&d_idx, T * sizeof(int32_t)));
        std::vector<float> lab(T);
        for (int t = 0; t < T; ++t) lab[t] = 1000.0f + 10.0f * t;
        HIP_OK(hipMemcpy(d_lab, lab.data(), T * sizeof(float), hipMemcpyHostToDevice));
        EXPECT(split_nn_set_scenarios(nn, d_dem, S, S, Q) == SPLIT_OK, "nn_set_scenarios");
        EXPECT(split_nn_set_norm(nn, 1000.0, 50.0) == SPLIT_OK, "nn_set_norm");
        EXPECT(split_nn_timing_enable(nn, 1) == SPLIT_OK, "nn_timing_enable");
        EXPECT(split_nn_predict(nn, d_tours, T, nt, d_pred, nullptr) == SPLIT_OK, "nn_predict");
        double nms = 0.0;
        int64_t nl = 0;
        EXPECT(split_nn_timing_get(nn, &nms, &nl) == SPLIT_OK && nl > 0, "nn_timing_get");
        EXPECT(split_nn_timing_reset(nn) == SPLIT_OK, "nn_timing_reset");
        std::vector<float> grad(SPLIT_NN_PARAMS), params(SPLIT_NN_PARAMS);
        double loss = 0.0;
        EXPECT(split_nn_gradient(nn, d_tours, d_lab, T, nt, grad.data(), &loss, nullptr) ==
                   SPLIT_OK, "nn_gradient");
        EXPECT(split_nn_train_step(nn, d_tours, d_lab, T, nt, 1e-3f, &loss, nullptr) == SPLIT_OK,
               "nn_train_step");
        double mean_loss = 0.0;
        EXPECT(split_nn_train(nn, d_tours, d_lab, T, nt, 4, 6, 1e-3f, 3, &mean_loss, nullptr) ==
                   SPLIT_OK, "nn_train");
        int64_t step = 0;
        EXPECT(split_nn_step(nn, &step) == SPLIT_OK && step == 7, "nn_step %lld",
               (long long)step);
        const std::string ck = scratch + "/host_sanitize_nn.ckpt";
        EXPECT(split_nn_save(nn, ck.c_str()) == SPLIT_OK, "nn_save");
        EXPECT(split_nn_params_get(nn, params.data()) == SPLIT_OK, "nn_params_get");
        EXPECT(split_nn_params_set(nn, params.data()) == SPLIT_OK, "nn_params_set");
        EXPECT(split_nn_load(nn, ck.c_str()) == SPLIT_OK, "nn_load");
        EXPECT(split_nn_load(nn, (scratch + "/no_such_file").c_str()) == SPLIT_E_INVAL,
               "nn_load missing");
        remove(ck.c_str());
        EXPECT(split_nn_shortlist(nn, d_tours, T, nt, 3, d_idx, d_pred, nullptr) == SPLIT_OK,
               "nn_shortlist");
        EXPECT(split_topk_smallest(ctx, d_pred, T, 2, d_idx, nullptr) == SPLIT_OK, "topk");
        std::vector<int32_t> sidx(3);
        std::vector<double> smean(3);
        int64_t best_idx = -1;
        double best_mean = 0.0;
        EXPECT(split_nn_screen(nn, d_tours, T, nt, 3, d_dem, S, S, Q, d_pred, sidx.data(),
                               smean.data(), &best_idx, &best_mean, nullptr) == SPLIT_OK,
               "nn_screen: %s", split_last_error(ctx));
        EXPECT(best_idx >= 0 && best_idx < T, "screen best index");

        // search with and without the surrogate
        std::vector<int32_t> best_tour(n);
        std::vector<double> tr_t(16), tr_m(16);
        int32_t tr_len = 0;
        split_search_result res{};
        EXPECT(split_search(ctx, nullptr, tour.data(), n, d_dem, S, S, Q, 8, 8, 10.0, 3, 11,
                            best_tour.data(), tr_t.data(), tr_m.data(), 16, &tr_len, &res,
                            nullptr) == SPLIT_OK, "search: %s", split_last_error(ctx));
        EXPECT(res.iterations == 3 && res.best_mean <= res.start_mean, "search result");
        EXPECT(split_search(ctx, nn, tour.data(), n, d_dem, S, S, Q, 4, 32, 10.0, 3, 12,
                            best_tour.data(), nullptr, nullptr, 0, nullptr, &res, nullptr) ==
                   SPLIT_OK, "search with the surrogate: %s", split_last_error(ctx));
        EXPECT(split_search(ctx, nullptr, tour.data(), n, d_dem, S, S, Q, 8, 16, 10.0, 3, 11,
                            best_tour.data(), nullptr, nullptr, 0, nullptr, &res, nullptr) ==
                   SPLIT_E_INVAL, "search pool != batch without a surrogate");
        split_nn_destroy(nn);
        HIP_OK(hipFree(d_tours));
        HIP_OK(hipFree(d_pred));
        HIP_OK(hipFree(d_lab));
        HIP_OK(hipFree(d_idx));
    }
    split_nn_destroy(nullptr);

    split_ctx_destroy(ctx);
    split_ctx_destroy(nullptr);
    HIP_OK(hipFree(d_dem));
    HIP_OK(hipFree(d_cost));
    HIP_OK(hipFree(d_cost2));
    if (g_fail) {
        fprintf(stderr, "host_sanitize_driver: %d check(s) failed\n", g_fail);
        return 1;
    }
    printf("host_sanitize_driver: all checks passed\n");
    return 0;
}
