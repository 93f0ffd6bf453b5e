// C-ABI host layer of libsplitgpu.so: argument checking, device buffers, kernel launches and
// the conversion of the exact device moments into the sample mean and variance.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <algorithm>
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

    // per-call device buffers, sized for the largest batch seen
    char *d_stage = nullptr;           // tours, tour offsets and work order of the call
    int64_t *d_rowoff = nullptr;
    uint32_t *d_rowoff32 = nullptr;
    int32_t *d_w = nullptr;
    int64_t cap_pos = 0;               // entries of the per-tour arrays
    int64_t cap_stage = 0;             // bytes of the staging buffers
    int32_t cap_T = 0;                 // tours
    unsigned long long *d_partials = nullptr;
    int64_t cap_partials = 0;
    DevStats *d_stats = nullptr;
    BatchCtl *d_ctl = nullptr;
    int lane_grid = 0;                 // persistent workgroups of the lane kernel

    // pinned host staging
    char *h_stage[kStages] = {};
    hipEvent_t stage_ev[kStages] = {};
    bool stage_ev_used[kStages] = {};
    int stage = 0;
    DevStats *h_stats = nullptr;
    hipEvent_t stats_ev = nullptr;
    bool have_call = false;
    int64_t last_S = 0;
    int32_t last_T = 0;

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

template <class P>
bool grow(P **ptr, size_t bytes)
{
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    return hipMalloc(ptr, bytes) == hipSuccess;
}

// Buffers for a batch of T tours with total_n positions, staging of stage_bytes and
// moment partials of T * nblocks blocks. Waits for enqueued work before replacing a buffer.
split_status ensure_capacity(split_ctx *ctx, int32_t T, int64_t total_n, int64_t stage_bytes,
                             int64_t partial_blocks)
{
    const int64_t pos = total_n + (int64_t)T * (1 + kRowPad);
    const bool g_pos = pos > ctx->cap_pos, g_stage = stage_bytes > ctx->cap_stage;
    const bool g_T = T > ctx->cap_T, g_part = partial_blocks > ctx->cap_partials;
    if (!g_pos && !g_stage && !g_T && !g_part) return SPLIT_OK;
    HIP_TRY(ctx, hipDeviceSynchronize());
    if (g_pos) {
        const int64_t np = pos < 4096 ? 4096 : pos + pos / 4;
        ctx->cap_pos = 0;
        if (!grow(&ctx->d_rowoff, sizeof(int64_t) * np) ||
            !grow(&ctx->d_rowoff32, sizeof(uint32_t) * np) || !grow(&ctx->d_w, sizeof(int32_t) * np))
            return fail(ctx, SPLIT_E_NOMEM, "device allocation for %lld tour positions failed",
                        (long long)np);
        ctx->cap_pos = np;
    }
    if (g_stage) {
        const int64_t nb = stage_bytes < 65536 ? 65536 : stage_bytes + stage_bytes / 4;
        ctx->cap_stage = 0;
        if (!grow(&ctx->d_stage, (size_t)nb))
            return fail(ctx, SPLIT_E_NOMEM, "device staging of %lld bytes failed", (long long)nb);
        for (int k = 0; k < kStages; ++k) {
            if (ctx->h_stage[k]) (void)hipHostFree(ctx->h_stage[k]);
            ctx->h_stage[k] = nullptr;
            ctx->stage_ev_used[k] = false;
            if (hipHostMalloc((void **)&ctx->h_stage[k], (size_t)nb, 0) != hipSuccess)
                return fail(ctx, SPLIT_E_NOMEM, "pinned staging of %lld bytes failed",
                            (long long)nb);
        }
        ctx->cap_stage = nb;
    }
    if (g_T) {
        const int32_t nt = T < 16 ? 16 : T;
        ctx->cap_T = 0;
        if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
        ctx->h_stats = nullptr;
        if (!grow(&ctx->d_stats, sizeof(DevStats) * nt) ||
            hipHostMalloc((void **)&ctx->h_stats, sizeof(DevStats) * nt, 0) != hipSuccess)
            return fail(ctx, SPLIT_E_NOMEM, "allocation of %d result blocks failed", nt);
        memset(ctx->h_stats, 0, sizeof(DevStats) * nt);
        ctx->cap_T = nt;
    }
    if (g_part) {
        ctx->cap_partials = 0;
        if (!grow(&ctx->d_partials, sizeof(unsigned long long) * 3 * partial_blocks))
            return fail(ctx, SPLIT_E_NOMEM, "allocation of moment partials failed");
        ctx->cap_partials = partial_blocks;
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
    hipDeviceProp_t prop;
    if (!g.ok || hipGetDeviceProperties(&prop, hip_device) != hipSuccess ||
        hipMalloc(&ctx->d_ctl, sizeof(BatchCtl)) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->stats_ev, hipEventDisableTiming) != hipSuccess) {
        split_ctx_destroy(ctx);
        return SPLIT_E_NOMEM;
    }
    // the lane kernel's LDS allows 8 workgroups per CU
    ctx->lane_grid = prop.multiProcessorCount * 8;
    for (int k = 0; k < kStages; ++k) {
        if (hipEventCreateWithFlags(&ctx->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
            split_ctx_destroy(ctx);
            return SPLIT_E_NOMEM;
        }
    }
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
        if (ctx->d_stage) (void)hipFree(ctx->d_stage);
        if (ctx->d_rowoff) (void)hipFree(ctx->d_rowoff);
        if (ctx->d_rowoff32) (void)hipFree(ctx->d_rowoff32);
        if (ctx->d_w) (void)hipFree(ctx->d_w);
        if (ctx->d_partials) (void)hipFree(ctx->d_partials);
        if (ctx->d_stats) (void)hipFree(ctx->d_stats);
        if (ctx->d_ctl) (void)hipFree(ctx->d_ctl);
        for (int k = 0; k < kStages; ++k) {
            if (ctx->h_stage[k]) (void)hipHostFree(ctx->h_stage[k]);
            if (ctx->stage_ev[k]) (void)hipEventDestroy(ctx->stage_ev[k]);
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

}  // extern "C"

namespace {

// The common path of split_eval and split_eval_batch.
split_status eval_batch(split_ctx *ctx, const char *who, const int32_t *tours,
                        const int64_t *tour_ptr, int32_t T, const int16_t *demand, int64_t S,
                        int64_t ld, int32_t Q, int32_t *cost, int64_t ldc, hipStream_t stream)
{
    if (ctx->kind < 0) return fail(ctx, SPLIT_E_INVAL, "%s: no instance set", who);
    if (!tours || !tour_ptr || !demand || !cost)
        return fail(ctx, SPLIT_E_INVAL, "%s: NULL pointer", who);
    if (T < 1) return fail(ctx, SPLIT_E_INVAL, "%s: need T >= 1", who);
    if (S < 1 || S > INT32_MAX || ld < S || ldc < S)
        return fail(ctx, SPLIT_E_INVAL, "%s: need 1 <= S < 2^31, ld >= S and ldc >= S", who);
    if (Q < 1 || Q > 16383) return fail(ctx, SPLIT_E_INVAL, "%s: need 1 <= Q <= 16383", who);
    if (tour_ptr[0] != 0) return fail(ctx, SPLIT_E_INVAL, "%s: tour_ptr[0] must be 0", who);
    int32_t max_id = 0, maxn = 0;
    for (int32_t t = 0; t < T; ++t) {
        const int64_t n64 = tour_ptr[t + 1] - tour_ptr[t];
        if (n64 < 1 || n64 > ctx->N)
            return fail(ctx, SPLIT_E_INVAL, "%s: tour %d has length %lld (need 1..N)", who, t,
                        (long long)n64);
        const int32_t n = (int32_t)n64;
        maxn = n > maxn ? n : maxn;
        const int32_t *tour = tours + tour_ptr[t];
        for (int32_t k = 0; k < n; ++k) {
            const int32_t c = tour[k];
            if (c < 1 || c > ctx->N || ctx->seen[c]) {
                for (int32_t j = 0; j < k; ++j) ctx->seen[tour[j]] = 0;
                return fail(ctx, SPLIT_E_TOUR, "%s: tour %d position %d: id %d is out of range "
                            "or repeated", who, t, k, c);
            }
            ctx->seen[c] = 1;
            max_id = c > max_id ? c : max_id;
        }
        for (int32_t k = 0; k < n; ++k) ctx->seen[tour[k]] = 0;
    }
    const int64_t total_n = tour_ptr[T];
    const int64_t nsb = (S + 63) / 64;
    if ((__int128)nsb * T >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_INVAL, "%s: T * ceil(S / 64) must be below 2^31", who);
    // |g| and |w| stay below (2n+3) * max_arc; keep them below 2^30 with a margin.
    if ((__int128)4 * ((__int128)maxn + 1) * ctx->max_arc >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_RANGE, "%s: 4*(n+1)*max_arc = 4*%d*%lld exceeds 2^31", who,
                    maxn + 1, (long long)ctx->max_arc);

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    // staging layout: tour offsets [T+1] int64, work order [T] int32, tours [total_n] int32
    const size_t off_order = sizeof(int64_t) * ((size_t)T + 1);
    const size_t off_tours = off_order + ((sizeof(int32_t) * (size_t)T + 7) & ~(size_t)7);
    const size_t stage_bytes = off_tours + sizeof(int32_t) * (size_t)total_n;
    const int32_t nblk = moment_blocks(S);
    split_status st = ensure_capacity(ctx, T, total_n, (int64_t)stage_bytes, (int64_t)nblk * T);
    if (st != SPLIT_OK) return st;

    // Upload through a pinned slot, reused only after its previous copy completed.
    const int slot = ctx->stage;
    ctx->stage = (ctx->stage + 1) % kStages;
    if (ctx->stage_ev_used[slot]) HIP_TRY(ctx, hipEventSynchronize(ctx->stage_ev[slot]));
    char *h = ctx->h_stage[slot];
    memcpy(h, tour_ptr, sizeof(int64_t) * ((size_t)T + 1));
    {
        // work order: longest tours first (ties by index), so short ones fill the tail
        int32_t *order = reinterpret_cast<int32_t *>(h + off_order);
        std::vector<int32_t> idx((size_t)T);
        for (int32_t t = 0; t < T; ++t) idx[t] = t;
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
            return tour_ptr[x + 1] - tour_ptr[x] > tour_ptr[y + 1] - tour_ptr[y];
        });
        memcpy(order, idx.data(), sizeof(int32_t) * (size_t)T);
    }
    memcpy(h + off_tours, tours, sizeof(int32_t) * (size_t)total_n);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_stage, h, stage_bytes, hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipEventRecord(ctx->stage_ev[slot], stream));
    ctx->stage_ev_used[slot] = true;

    TourDev td;
    td.tptr = reinterpret_cast<const int64_t *>(ctx->d_stage);
    td.order = reinterpret_cast<const int32_t *>(ctx->d_stage + off_order);
    td.tours = reinterpret_cast<const int32_t *>(ctx->d_stage + off_tours);
    td.T = T;
    td.rowoff = ctx->d_rowoff;
    td.rowoff32 = ctx->d_rowoff32;
    td.w = ctx->d_w;

    PrepArgs pa;
    pa.tour = td;
    pa.N = ctx->N;
    pa.kind = ctx->kind;
    pa.xy = ctx->d_xy;
    pa.dist = ctx->d_dist;
    pa.ld = ld;
    pa.stats = ctx->d_stats;
    pa.ctl = ctx->d_ctl;
    HIP_TRY(ctx, launch_prep(pa, stream));

    EvalArgs ea;
    ea.demand = reinterpret_cast<const uint16_t *>(demand);
    ea.ld = ld;
    ea.S = S;
    ea.Q = Q;
    ea.tour = td;
    ea.cost = cost;
    ea.ldc = ldc;
    ea.stats = ctx->d_stats;
    ea.ctl = ctx->d_ctl;
    ea.maxn = maxn;

    int form = ctx->form;
    if (form == SPLIT_FORM_AUTO) form = S <= kWaveAutoMaxS ? SPLIT_FORM_WAVE : SPLIT_FORM_LANE;
    // The lane kernel addresses demands with 32-bit buffer offsets.
    const __int128 lane_bytes = ((__int128)(max_id - 1) * ld + S) * 2;
    const bool lane_addressable = lane_bytes <= (__int128)kRowAbsent;
    ea.lane_bytes = lane_addressable ? (uint32_t)lane_bytes : 0u;
    if (form == SPLIT_FORM_LANE && !lane_addressable) form = SPLIT_FORM_WAVE;
    const int64_t items = nsb * T;
    ea.lane_grid = (int32_t)(items < ctx->lane_grid ? items : ctx->lane_grid);
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
    ma.ldc = ldc;
    ma.S = S;
    ma.T = T;
    ma.partials = ctx->d_partials;
    ma.nblocks = nblk;
    ma.stats = ctx->d_stats;
    HIP_TRY(ctx, launch_moments(ma, stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_stats, ctx->d_stats, sizeof(DevStats) * (size_t)T,
                                hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipEventRecord(ctx->stats_ev, stream));
    ctx->have_call = true;
    ctx->last_S = S;
    ctx->last_T = T;
    return SPLIT_OK;
}

}  // namespace

extern "C" {

split_status split_eval(split_ctx *ctx, const int32_t *tour, int32_t n, const int16_t *demand,
                        int64_t S, int64_t ld, int32_t Q, int32_t *cost, split_stats *stats,
                        void *hip_stream)
{
    if (!ctx) return SPLIT_E_INVAL;
    const int64_t tour_ptr[2] = {0, n};
    split_status st = eval_batch(ctx, "split_eval", tour, tour_ptr, 1, demand, S, ld, Q, cost, S,
                                 (hipStream_t)hip_stream);
    if (st != SPLIT_OK) return st;
    if (stats) return split_stats_get(ctx, stats);
    return SPLIT_OK;
}

split_status split_eval_batch(split_ctx *ctx, const int32_t *tours, const int64_t *tour_ptr,
                              int32_t T, const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                              int32_t *cost, int64_t ldc, split_stats *stats,
                              int32_t *tour_status, void *hip_stream)
{
    if (!ctx) return SPLIT_E_INVAL;
    split_status st = eval_batch(ctx, "split_eval_batch", tours, tour_ptr, T, demand, S, ld, Q,
                                 cost, ldc, (hipStream_t)hip_stream);
    if (st != SPLIT_OK) return st;
    if (stats || tour_status) return split_batch_stats_get(ctx, stats, tour_status);
    return SPLIT_OK;
}

split_status split_batch_stats_get(split_ctx *ctx, split_stats *stats, int32_t *tour_status)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!ctx->have_call) return fail(ctx, SPLIT_E_INVAL, "split_batch_stats_get: no evaluation yet");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, hipEventSynchronize(ctx->stats_ev));
    int bad = -1;
    for (int32_t t = 0; t < ctx->last_T; ++t) {
        const DevStats &d = ctx->h_stats[t];
        if (stats) fill_stats(d, ctx->last_S, stats + t);
        if (tour_status) tour_status[t] = d.err_demand ? SPLIT_E_DEMAND : SPLIT_OK;
        if (d.err_demand && bad < 0) bad = t;
    }
    if (bad >= 0)
        return fail(ctx, SPLIT_E_DEMAND, "tour %d: a scenario has a demand q < 0 or q > Q on the "
                    "tour", bad);
    return SPLIT_OK;
}

split_status split_stats_get(split_ctx *ctx, split_stats *stats)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!stats) return fail(ctx, SPLIT_E_INVAL, "split_stats_get: NULL stats");
    if (!ctx->have_call) return fail(ctx, SPLIT_E_INVAL, "split_stats_get: no evaluation yet");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, hipEventSynchronize(ctx->stats_ev));
    const DevStats d = ctx->h_stats[0];
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
