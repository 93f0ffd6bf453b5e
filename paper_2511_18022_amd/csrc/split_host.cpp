// C-ABI host layer of libsplitgpu.so: argument checking, device buffers, kernel launches and
// the conversion of the exact device moments into the sample mean and variance.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/split.h"
#include "split_internal.h"

using namespace splitgpu;

namespace {

constexpr int kStages = 8;              // pinned host slots for tour uploads
constexpr int64_t kWaveAutoMaxS = 4096;  // SPLIT_FORM_AUTO uses the wave form up to this S
constexpr int kMaxTimingPairs = 4096;

}  // namespace

struct split_ctx {
    int device = 0;
    std::string err;
    int form = SPLIT_FORM_AUTO;

    // instance
    int32_t N = 0;
    int kind = -1;  // 0 coordinates, 1 matrix
    int32_t *d_xy = nullptr;
    int32_t *d_dist = nullptr;
    int64_t max_arc = 0;
    std::vector<unsigned char> seen;

    // per-call device buffers
    int32_t *d_tour = nullptr;
    int64_t *d_rowoff = nullptr;
    uint32_t *d_rowoff32 = nullptr;
    int32_t *d_w = nullptr;
    int32_t cap_n = 0;
    int32_t *d_ovf = nullptr;
    int64_t cap_S = 0;
    unsigned long long *d_partials = nullptr;
    DevStats *d_stats = nullptr;

    // pinned host staging
    int32_t *h_tour[kStages] = {};
    hipEvent_t tour_ev[kStages] = {};
    bool tour_ev_used[kStages] = {};
    int stage = 0;
    DevStats *h_stats = nullptr;
    hipEvent_t stats_ev = nullptr;
    bool have_call = false;
    int64_t last_S = 0;

    // timing of the dominant kernel
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tpairs;
    size_t tpairs_used = 0;
    double ms_acc = 0.0;
    int64_t launches = 0;
    const char *tname = "";
};

namespace {

split_status fail(split_ctx *ctx, split_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

split_status hip_fail(split_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, SPLIT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// Makes ctx->device current for the scope of one API call and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

void free_instance(split_ctx *ctx)
{
    if (ctx->d_xy) (void)hipFree(ctx->d_xy);
    if (ctx->d_dist) (void)hipFree(ctx->d_dist);
    ctx->d_xy = nullptr;
    ctx->d_dist = nullptr;
    ctx->N = 0;
    ctx->kind = -1;
    ctx->max_arc = 0;
}

split_status ensure_capacity(split_ctx *ctx, int32_t n, int64_t S)
{
    const bool grow_n = n > ctx->cap_n;
    const bool grow_S = S > ctx->cap_S;
    if (!grow_n && !grow_S) return SPLIT_OK;
    // Buffers may still be used by enqueued work: wait before replacing them.
    HIP_TRY(ctx, hipDeviceSynchronize());
    if (grow_n) {
        int32_t nn = n < 1024 ? 1024 : n;
        if (ctx->d_tour) (void)hipFree(ctx->d_tour);
        if (ctx->d_rowoff) (void)hipFree(ctx->d_rowoff);
        if (ctx->d_rowoff32) (void)hipFree(ctx->d_rowoff32);
        if (ctx->d_w) (void)hipFree(ctx->d_w);
        ctx->d_tour = nullptr;
        ctx->d_rowoff = nullptr;
        ctx->d_rowoff32 = nullptr;
        ctx->d_w = nullptr;
        ctx->cap_n = 0;
        if (hipMalloc(&ctx->d_tour, sizeof(int32_t) * nn) != hipSuccess ||
            hipMalloc(&ctx->d_rowoff, sizeof(int64_t) * (nn + 1 + kRowPad)) != hipSuccess ||
            hipMalloc(&ctx->d_rowoff32, sizeof(uint32_t) * (nn + 1 + kRowPad)) != hipSuccess ||
            hipMalloc(&ctx->d_w, sizeof(int32_t) * (nn + 1 + kRowPad)) != hipSuccess)
            return fail(ctx, SPLIT_E_NOMEM, "device allocation for n=%d failed", nn);
        for (int k = 0; k < kStages; ++k) {
            if (ctx->h_tour[k]) (void)hipHostFree(ctx->h_tour[k]);
            ctx->h_tour[k] = nullptr;
            if (hipHostMalloc((void **)&ctx->h_tour[k], sizeof(int32_t) * nn, 0) != hipSuccess)
                return fail(ctx, SPLIT_E_NOMEM, "pinned allocation for n=%d failed", nn);
        }
        ctx->cap_n = nn;
    }
    if (grow_S) {
        int64_t ss = S < 65536 ? 65536 : S;
        if (ctx->d_ovf) (void)hipFree(ctx->d_ovf);
        ctx->d_ovf = nullptr;
        ctx->cap_S = 0;
        if (hipMalloc(&ctx->d_ovf, sizeof(int32_t) * ss) != hipSuccess)
            return fail(ctx, SPLIT_E_NOMEM, "device allocation for S=%lld failed", (long long)ss);
        ctx->cap_S = ss;
    }
    return SPLIT_OK;
}

split_status collect_timing(split_ctx *ctx)
{
    for (size_t k = 0; k < ctx->tpairs_used; ++k) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->tpairs[k].second));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->tpairs[k].first, ctx->tpairs[k].second));
        ctx->ms_acc += ms;
        ctx->launches += 1;
    }
    ctx->tpairs_used = 0;
    return SPLIT_OK;
}

split_status timing_begin(split_ctx *ctx, hipStream_t stream, hipEvent_t *stop_out)
{
    *stop_out = nullptr;
    if (!ctx->timing) return SPLIT_OK;
    if (ctx->tpairs_used == (size_t)kMaxTimingPairs) {
        split_status st = collect_timing(ctx);
        if (st != SPLIT_OK) return st;
    }
    if (ctx->tpairs_used == ctx->tpairs.size()) {
        hipEvent_t a, b;
        HIP_TRY(ctx, hipEventCreate(&a));
        HIP_TRY(ctx, hipEventCreate(&b));
        ctx->tpairs.emplace_back(a, b);
    }
    auto &pr = ctx->tpairs[ctx->tpairs_used++];
    HIP_TRY(ctx, hipEventRecord(pr.first, stream));
    *stop_out = pr.second;
    return SPLIT_OK;
}

void fill_stats(const DevStats &d, int64_t S, split_stats *out)
{
    out->sum = (int64_t)d.sum;
    out->sumsq_lo = d.sq_lo;
    out->sumsq_hi = d.sq_hi;
    out->mean = (double)(int64_t)d.sum / (double)S;
    if (S == 1) {
        out->var = 0.0;
    } else {
        const unsigned __int128 sq = ((unsigned __int128)d.sq_hi << 64) | d.sq_lo;
        const unsigned __int128 sm = d.sum;
        const unsigned __int128 num = (unsigned __int128)(uint64_t)S * sq - sm * sm;
        out->var = ((double)num / (double)S) / (double)(S - 1);
    }
    out->n_fallback = d.ovf_count;
}

}  // namespace

extern "C" {

split_status split_ctx_create(int hip_device, split_ctx **out)
{
    if (!out) return SPLIT_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
        return SPLIT_E_INVAL;
    split_ctx *ctx = new (std::nothrow) split_ctx();
    if (!ctx) return SPLIT_E_NOMEM;
    ctx->device = hip_device;
    DeviceGuard g(hip_device);
    if (!g.ok || hipMalloc(&ctx->d_stats, sizeof(DevStats)) != hipSuccess ||
        hipMalloc(&ctx->d_partials, sizeof(unsigned long long) * 3 * 1024) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_stats, sizeof(DevStats), 0) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->stats_ev, hipEventDisableTiming) != hipSuccess) {
        split_ctx_destroy(ctx);
        return SPLIT_E_NOMEM;
    }
    for (int k = 0; k < kStages; ++k) {
        if (hipEventCreateWithFlags(&ctx->tour_ev[k], hipEventDisableTiming) != hipSuccess) {
            split_ctx_destroy(ctx);
            return SPLIT_E_NOMEM;
        }
    }
    memset(ctx->h_stats, 0, sizeof(DevStats));
    *out = ctx;
    return SPLIT_OK;
}

void split_ctx_destroy(split_ctx *ctx)
{
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        free_instance(ctx);
        if (ctx->d_tour) (void)hipFree(ctx->d_tour);
        if (ctx->d_rowoff) (void)hipFree(ctx->d_rowoff);
        if (ctx->d_rowoff32) (void)hipFree(ctx->d_rowoff32);
        if (ctx->d_w) (void)hipFree(ctx->d_w);
        if (ctx->d_ovf) (void)hipFree(ctx->d_ovf);
        if (ctx->d_partials) (void)hipFree(ctx->d_partials);
        if (ctx->d_stats) (void)hipFree(ctx->d_stats);
        for (int k = 0; k < kStages; ++k) {
            if (ctx->h_tour[k]) (void)hipHostFree(ctx->h_tour[k]);
            if (ctx->tour_ev[k]) (void)hipEventDestroy(ctx->tour_ev[k]);
        }
        if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
        if (ctx->stats_ev) (void)hipEventDestroy(ctx->stats_ev);
        for (auto &pr : ctx->tpairs) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    }
    delete ctx;
}

const char *split_last_error(const split_ctx *ctx)
{
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

split_status split_instance_set_coords(split_ctx *ctx, int32_t N, const int32_t *xy)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!xy || N < 1 || N > SPLIT_MAX_N)
        return fail(ctx, SPLIT_E_INVAL, "set_coords: need xy != NULL and 1 <= N <= %d", SPLIT_MAX_N);
    int64_t lo[2] = {INT64_MAX, INT64_MAX}, hi[2] = {INT64_MIN, INT64_MIN};
    for (int64_t v = 0; v <= N; ++v)
        for (int c = 0; c < 2; ++c) {
            const int64_t x = xy[2 * v + c];
            if (x < -(1 << 20) || x > (1 << 20))
                return fail(ctx, SPLIT_E_INVAL, "set_coords: |coordinate| must be <= 2^20");
            lo[c] = x < lo[c] ? x : lo[c];
            hi[c] = x > hi[c] ? x : hi[c];
        }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    HIP_TRY(ctx, hipDeviceSynchronize());
    free_instance(ctx);
    HIP_TRY(ctx, hipMalloc(&ctx->d_xy, sizeof(int32_t) * 2 * ((size_t)N + 1)));
    HIP_TRY(ctx, hipMemcpy(ctx->d_xy, xy, sizeof(int32_t) * 2 * ((size_t)N + 1),
                           hipMemcpyHostToDevice));
    const double dx = (double)(hi[0] - lo[0]), dy = (double)(hi[1] - lo[1]);
    ctx->max_arc = (int64_t)ceil(sqrt(dx * dx + dy * dy)) + 1;  // bound on any rounded distance
    ctx->N = N;
    ctx->kind = 0;
    ctx->seen.assign((size_t)N + 1, 0);
    return SPLIT_OK;
}

split_status split_instance_set_dist(split_ctx *ctx, int32_t N, const int32_t *d)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!d || N < 1 || N > SPLIT_MAX_N)
        return fail(ctx, SPLIT_E_INVAL, "set_dist: need d != NULL and 1 <= N <= %d", SPLIT_MAX_N);
    const size_t V = (size_t)N + 1;
    int64_t mx = 0;
    for (size_t k = 0; k < V * V; ++k) {
        if (d[k] < 0) return fail(ctx, SPLIT_E_INVAL, "set_dist: negative entry at %zu", k);
        mx = d[k] > mx ? d[k] : mx;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    HIP_TRY(ctx, hipDeviceSynchronize());
    free_instance(ctx);
    HIP_TRY(ctx, hipMalloc(&ctx->d_dist, sizeof(int32_t) * V * V));
    HIP_TRY(ctx, hipMemcpy(ctx->d_dist, d, sizeof(int32_t) * V * V, hipMemcpyHostToDevice));
    ctx->max_arc = mx;
    ctx->N = N;
    ctx->kind = 1;
    ctx->seen.assign(V, 0);
    return SPLIT_OK;
}

split_status split_eval(split_ctx *ctx, const int32_t *tour, int32_t n, const int16_t *demand,
                        int64_t S, int64_t ld, int32_t Q, int32_t *cost, split_stats *stats,
                        void *hip_stream)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (ctx->kind < 0) return fail(ctx, SPLIT_E_INVAL, "split_eval: no instance set");
    if (!tour || !demand || !cost) return fail(ctx, SPLIT_E_INVAL, "split_eval: NULL pointer");
    if (n < 1 || n > ctx->N) return fail(ctx, SPLIT_E_INVAL, "split_eval: need 1 <= n <= N");
    if (S < 1 || S > INT32_MAX || ld < S)
        return fail(ctx, SPLIT_E_INVAL, "split_eval: need 1 <= S < 2^31 and ld >= S");
    if (Q < 1 || Q > 16383) return fail(ctx, SPLIT_E_INVAL, "split_eval: need 1 <= Q <= 16383");
    int32_t max_id = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t c = tour[k];
        max_id = c > max_id ? c : max_id;
        if (c < 1 || c > ctx->N || ctx->seen[c]) {
            for (int32_t j = 0; j < k; ++j) ctx->seen[tour[j]] = 0;
            return fail(ctx, SPLIT_E_TOUR, "split_eval: tour[%d]=%d is out of range or repeated",
                        k, c);
        }
        ctx->seen[c] = 1;
    }
    for (int32_t k = 0; k < n; ++k) ctx->seen[tour[k]] = 0;
    // |g| and |w| stay below (2n+3) * max_arc; keep them below 2^30 with a margin.
    if ((__int128)4 * ((__int128)n + 1) * ctx->max_arc >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_RANGE, "split_eval: 4*(n+1)*max_arc = 4*%d*%lld exceeds 2^31",
                    n + 1, (long long)ctx->max_arc);

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    hipStream_t stream = (hipStream_t)hip_stream;
    split_status st = ensure_capacity(ctx, n, S);
    if (st != SPLIT_OK) return st;

    // Tour upload through a pinned slot, reused only after its previous copy completed.
    const int slot = ctx->stage;
    ctx->stage = (ctx->stage + 1) % kStages;
    if (ctx->tour_ev_used[slot]) HIP_TRY(ctx, hipEventSynchronize(ctx->tour_ev[slot]));
    memcpy(ctx->h_tour[slot], tour, sizeof(int32_t) * (size_t)n);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_tour, ctx->h_tour[slot], sizeof(int32_t) * (size_t)n,
                                hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipEventRecord(ctx->tour_ev[slot], stream));
    ctx->tour_ev_used[slot] = true;

    PrepArgs pa;
    pa.tour = ctx->d_tour;
    pa.n = n;
    pa.N = ctx->N;
    pa.kind = ctx->kind;
    pa.xy = ctx->d_xy;
    pa.dist = ctx->d_dist;
    pa.ld = ld;
    pa.out.rowoff = ctx->d_rowoff;
    pa.out.rowoff32 = ctx->d_rowoff32;
    pa.out.w = ctx->d_w;
    pa.stats = ctx->d_stats;
    HIP_TRY(ctx, launch_prep(pa, stream));

    EvalArgs ea;
    ea.demand = reinterpret_cast<const uint16_t *>(demand);
    ea.ld = ld;
    ea.S = S;
    ea.n = n;
    ea.Q = Q;
    ea.tour = pa.out;
    ea.cost = cost;
    ea.stats = ctx->d_stats;
    ea.ovf_list = ctx->d_ovf;

    int form = ctx->form;
    if (form == SPLIT_FORM_AUTO) form = S <= kWaveAutoMaxS ? SPLIT_FORM_WAVE : SPLIT_FORM_LANE;
    // The lane kernel addresses demands with 32-bit buffer offsets.
    const __int128 lane_bytes = ((__int128)(max_id - 1) * ld + S) * 2;
    const bool lane_addressable = lane_bytes <= (__int128)kRowAbsent;
    ea.lane_bytes = lane_addressable ? (uint32_t)lane_bytes : 0u;
    if (form == SPLIT_FORM_LANE && !lane_addressable) form = SPLIT_FORM_WAVE;
    hipEvent_t stop = nullptr;
    st = timing_begin(ctx, stream, &stop);
    if (st != SPLIT_OK) return st;
    if (form == SPLIT_FORM_WAVE) {
        ctx->tname = wave_kernel_name();
        HIP_TRY(ctx, launch_wave_all(ea, stream));
        if (stop) HIP_TRY(ctx, hipEventRecord(stop, stream));
    } else {
        ctx->tname = lane_kernel_name();
        HIP_TRY(ctx, launch_lane(ea, stream));
        if (stop) HIP_TRY(ctx, hipEventRecord(stop, stream));
        HIP_TRY(ctx, launch_wave_fallback(ea, stream));
    }

    MomentArgs ma;
    ma.cost = cost;
    ma.S = S;
    ma.partials = ctx->d_partials;
    ma.nblocks = moment_blocks(S);
    ma.stats = ctx->d_stats;
    HIP_TRY(ctx, launch_moments(ma, stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_stats, ctx->d_stats, sizeof(DevStats),
                                hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipEventRecord(ctx->stats_ev, stream));
    ctx->have_call = true;
    ctx->last_S = S;
    if (stats) return split_stats_get(ctx, stats);
    return SPLIT_OK;
}

split_status split_stats_get(split_ctx *ctx, split_stats *stats)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!stats) return fail(ctx, SPLIT_E_INVAL, "split_stats_get: NULL stats");
    if (!ctx->have_call) return fail(ctx, SPLIT_E_INVAL, "split_stats_get: no evaluation yet");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, hipEventSynchronize(ctx->stats_ev));
    const DevStats d = *ctx->h_stats;
    fill_stats(d, ctx->last_S, stats);
    if (d.err_demand)
        return fail(ctx, SPLIT_E_DEMAND,
                    "split_eval: a scenario has a demand q < 0 or q > Q on the tour");
    return SPLIT_OK;
}

split_status split_set_form(split_ctx *ctx, int form)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (form != SPLIT_FORM_AUTO && form != SPLIT_FORM_LANE && form != SPLIT_FORM_WAVE)
        return fail(ctx, SPLIT_E_INVAL, "split_set_form: unknown form %d", form);
    ctx->form = form;
    return SPLIT_OK;
}

split_status split_timing_enable(split_ctx *ctx, int enable)
{
    if (!ctx) return SPLIT_E_INVAL;
    ctx->timing = enable != 0;
    return SPLIT_OK;
}

split_status split_timing_get(split_ctx *ctx, double *ms_total, int64_t *launches,
                              const char **kernel_name)
{
    if (!ctx) return SPLIT_E_INVAL;
    DeviceGuard g(ctx->device);
    split_status st = collect_timing(ctx);
    if (st != SPLIT_OK) return st;
    if (ms_total) *ms_total = ctx->ms_acc;
    if (launches) *launches = ctx->launches;
    if (kernel_name) *kernel_name = ctx->tname;
    return SPLIT_OK;
}

split_status split_timing_reset(split_ctx *ctx)
{
    if (!ctx) return SPLIT_E_INVAL;
    DeviceGuard g(ctx->device);
    split_status st = collect_timing(ctx);
    ctx->ms_acc = 0.0;
    ctx->launches = 0;
    return st;
}

}  // extern "C"
