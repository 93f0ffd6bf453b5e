// Local search over giant tours with the scenario-batched Split as the objective
// (include/split_search.h). Built on the library's public C ABI: captured graphs for the exact
// evaluation of each batch of neighbours, the surrogate and top-k to shortlist a larger pool.
#include <hip/hip_runtime.h>

#include <string.h>

#include <chrono>
#include <vector>

#include "../../include/split_search.h"
#include "nn_internal.h"
#include "split_internal.h"

using namespace splitgpu;

namespace {

uint64_t next_u64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One random move for a tour of n >= 2 positions: (0, i, j) a 2-opt reversal of positions
// min(i,j)..max(i,j), (1, i, j) a relocation of the customer at i to position j; i != j.
void draw_move(int32_t n, uint64_t &rs, int32_t *mv)
{
    const uint64_t r = next_u64(rs);
    const int32_t i = (int32_t)((r & 0xFFFFFFFFull) % (uint64_t)n);
    int32_t j = (int32_t)((r >> 32) % (uint64_t)(n - 1));
    if (j >= i) ++j;
    mv[0] = (next_u64(rs) & 1) ? 0 : 1;
    mv[1] = i;
    mv[2] = j;
}

// cur with move mv applied, written to out (the host twin of the device move kernel)
void apply_move(const int32_t *cur, int32_t n, const int32_t *mv, int32_t *out)
{
    memcpy(out, cur, sizeof(int32_t) * (size_t)n);
    const int32_t i = mv[1], j = mv[2];
    if (mv[0] == 0) {
        // 2-opt: reverse positions lo..hi
        int32_t lo = i < j ? i : j, hi = i < j ? j : i;
        for (; lo < hi; ++lo, --hi) {
            const int32_t t = out[lo];
            out[lo] = out[hi];
            out[hi] = t;
        }
    } else {
        // relocate: the customer at position i moves to position j
        const int32_t x = out[i];
        if (i < j)
            memmove(out + i, out + i + 1, sizeof(int32_t) * (size_t)(j - i));
        else
            memmove(out + j + 1, out + j, sizeof(int32_t) * (size_t)(i - j));
        out[j] = x;
    }
}

struct SearchBuffers {
    int32_t *cost = nullptr, *dcand = nullptr, *didx = nullptr, *dcur = nullptr;
    int32_t *dmoves = nullptr, *dsel = nullptr;
    split_graph *graph = nullptr;
    ~SearchBuffers()
    {
        split_graph_destroy(graph);
        for (int32_t *p : {cost, dcand, didx, dcur, dmoves, dsel})
            if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" split_status split_search(split_ctx *ctx, split_nn *nn, const int32_t *tour0,
                                     int32_t n, const int16_t *demand, int64_t S, int64_t ld,
                                     int32_t Q, int32_t batch, int32_t pool, double budget_s,
                                     int64_t max_iters, uint64_t seed, int32_t *best_tour,
                                     double *trace_t, double *trace_mean, int32_t trace_cap,
                                     int32_t *trace_len, split_search_result *result,
                                     void *hip_stream)
{
    if (!ctx) return SPLIT_E_INVAL;
    int32_t N = 0;
    int kind = 0;
    const int32_t *xy = nullptr, *dist = nullptr;
    int64_t max_arc = 0;
    if (!ctx_instance(ctx, &N, &kind, &xy, &dist, &max_arc))
        return ctx_fail(ctx, SPLIT_E_INVAL, "split_search: no instance set");
    if (!tour0 || !best_tour || !demand || n < 1 || n > N || batch < 1 || batch > 4096 ||
        pool < batch || pool > 65536 || (!nn && pool != batch) || !(budget_s >= 0.0) ||
        max_iters < 0 || trace_cap < 0)
        return ctx_fail(ctx, SPLIT_E_INVAL, "split_search: need tour0, best_tour, demand, "
                        "1 <= n <= N, 1 <= batch <= 4096, batch <= pool <= 65536 (pool == batch "
                        "without a surrogate), budget_s >= 0, max_iters >= 0");
    std::vector<unsigned char> seen((size_t)N + 1, 0);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t c = tour0[k];
        if (c < 1 || c > N || seen[c])
            return ctx_fail(ctx, SPLIT_E_TOUR, "split_search: start tour position %d: id %d is "
                            "out of range or repeated", k, c);
        seen[c] = 1;
    }
    struct Restore {
        int prev = -1;
        ~Restore()
        {
            if (prev >= 0) (void)hipSetDevice(prev);
        }
    } restore;
    if (hipGetDevice(&restore.prev) != hipSuccess) restore.prev = -1;
    if (hipSetDevice(ctx_device(ctx)) != hipSuccess)
        return ctx_fail(ctx, SPLIT_E_HIP, "split_search: hipSetDevice failed");
    hipStream_t st = (hipStream_t)hip_stream;
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&]() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };

    SearchBuffers b;
    if (hipMalloc(&b.cost, sizeof(int32_t) * (size_t)batch * (size_t)S) != hipSuccess)
        return ctx_fail(ctx, SPLIT_E_NOMEM, "split_search: cost buffer");
    if (nn && (hipMalloc(&b.dcand, sizeof(int32_t) * (size_t)pool * n) != hipSuccess ||
               hipMalloc(&b.didx, sizeof(int32_t) * (size_t)batch) != hipSuccess ||
               hipMalloc(&b.dcur, sizeof(int32_t) * (size_t)n) != hipSuccess ||
               hipMalloc(&b.dmoves, sizeof(int32_t) * 3 * (size_t)pool) != hipSuccess ||
               hipMalloc(&b.dsel, sizeof(int32_t) * (size_t)batch * n) != hipSuccess))
        return ctx_fail(ctx, SPLIT_E_NOMEM, "split_search: surrogate buffers");
    split_status s = split_graph_create(ctx, batch, (int64_t)batch * n, demand, S, ld, Q, b.cost, S,
                                        &b.graph);
    if (s != SPLIT_OK) return s;

    std::vector<int32_t> cur(tour0, tour0 + n), sel((size_t)batch * n);
    std::vector<int32_t> moves(3 * (size_t)pool);
    std::vector<int64_t> ptr((size_t)batch + 1);
    std::vector<split_stats> stats((size_t)batch);
    std::vector<int32_t> status((size_t)batch);
    split_search_result res = {};
    int32_t tl = 0;
    auto record = [&](double t, double m) {
        if (tl < trace_cap) {
            if (trace_t) trace_t[tl] = t;
            if (trace_mean) trace_mean[tl] = m;
        }
        ++tl;
    };
    // the start tour
    const int64_t p1[2] = {0, n};
    s = split_graph_launch(b.graph, cur.data(), p1, 1, st);
    if (s == SPLIT_OK) s = split_graph_stats(b.graph, stats.data(), status.data());
    if (s != SPLIT_OK) return s;
    double cur_mean = stats[0].mean;
    res.start_mean = cur_mean;
    res.evaluated = 1;
    record(elapsed(), cur_mean);
    for (int32_t t = 0; t <= batch; ++t) ptr[t] = (int64_t)t * n;
    uint64_t rs = seed;
    while (n >= 2 && res.iterations < max_iters && elapsed() < budget_s) {
        for (int32_t c = 0; c < pool; ++c) draw_move(n, rs, moves.data() + 3 * (size_t)c);
        if (nn) {
            // candidates built on the device from the incumbent and the moves, predicted, and
            // the shortlist gathered there; only the batch comes back for exact evaluation
            if (hipMemcpyAsync(b.dcur, cur.data(), sizeof(int32_t) * (size_t)n,
                               hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(b.dmoves, moves.data(), sizeof(int32_t) * 3 * (size_t)pool,
                               hipMemcpyHostToDevice, st) != hipSuccess ||
                nn_launch_moves(b.dcur, b.dmoves, pool, n, b.dcand, st) != hipSuccess)
                return ctx_fail(ctx, SPLIT_E_HIP, "split_search: building the candidates failed");
            s = split_nn_shortlist(nn, b.dcand, pool, n, batch, b.didx, nullptr, hip_stream);
            if (s != SPLIT_OK) return s;
            if (nn_launch_gather(b.dcand, nullptr, b.didx, batch, n, b.dsel, nullptr, st) !=
                    hipSuccess ||
                hipMemcpyAsync(sel.data(), b.dsel, sizeof(int32_t) * (size_t)batch * n,
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return ctx_fail(ctx, SPLIT_E_HIP, "split_search: shortlist copy failed");
            res.predicted += pool;
        } else {
            for (int32_t c = 0; c < batch; ++c)
                apply_move(cur.data(), n, moves.data() + 3 * (size_t)c, sel.data() + (size_t)c * n);
        }
        const int32_t *eval = sel.data();
        s = split_graph_launch(b.graph, eval, ptr.data(), batch, st);
        if (s == SPLIT_OK) s = split_graph_stats(b.graph, stats.data(), status.data());
        if (s != SPLIT_OK) return s;
        res.evaluated += batch;
        res.iterations += 1;
        int32_t bk = 0;
        for (int32_t k = 1; k < batch; ++k)
            if (stats[k].mean < stats[bk].mean) bk = k;
        if (stats[bk].mean < cur_mean) {
            cur_mean = stats[bk].mean;
            memcpy(cur.data(), eval + (size_t)bk * n, sizeof(int32_t) * (size_t)n);
            res.improvements += 1;
            record(elapsed(), cur_mean);
        }
    }
    memcpy(best_tour, cur.data(), sizeof(int32_t) * (size_t)n);
    res.best_mean = cur_mean;
    res.seconds = elapsed();
    if (trace_len) *trace_len = tl < trace_cap ? tl : trace_cap;
    if (result) *result = res;
    return SPLIT_OK;
}
