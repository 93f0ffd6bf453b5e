// C-ABI host layer of libsplitgpu.so: argument checking, device buffers, kernel launches, the
// autotuner, captured evaluation graphs, and the conversion of the exact device moments into
// the sample mean and variance.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "split_internal.h"

using namespace splitgpu;

namespace {

constexpr int kStages = 8;              // pinned host slots for tour uploads
// SPLIT_FORM_AUTO takes the wave form for short tours over few scenarios, where the lane
// kernel's per-item prologue outweighs its per-state advantage. Measured crossover of whole
// evaluations (tours of 8..256 positions): the wave form is ahead up to n = 32 at S = 256, up to
// n = 24 at S = 1024 and up to n = 16 at S = 4096; the lane form everywhere else (at n = 1000
// from S = 1024 on, at 2.6x and more).
bool auto_wave(int64_t S, int32_t maxn)
{
    if (S <= 256) return maxn <= 32;
    if (S <= 1024) return maxn <= 24;
    if (S <= 4096) return maxn <= 16;
    return false;
}
// The lane kernel compares load differences in 16 bits, exact while 8 * max(q) + Q < 2^15;
// evaluations with a larger capacity run in the wave form, which is exact for any Q.
constexpr int32_t kLaneMaxQ = 16383;
constexpr int kMaxTimingPairs = 4096;
constexpr int kGraphSlots = 2;          // a graph's launches alternate between two host slots
constexpr int32_t kMaxLanePerCu = 8;    // the lane kernel's LDS allows 8 workgroups per CU
constexpr int32_t kLaneStaticPerCu = kMaxLanePerCu;  // fixed-stride grid: all resident at once
constexpr int64_t kLaneStaticMaxRounds = 16;         // and at most this many items each

// Device buffers of one evaluation sequence. The context's grow with its calls; a graph owns
// a fixed set.
struct EvalBuffers {
    char *d_stage = nullptr;  // staged header, see TourDev
    int64_t cap_stage = 0;
    int64_t *d_rowoff = nullptr;
    uint32_t *d_rowoff32 = nullptr;
    int32_t *d_w = nullptr;
    int64_t cap_pos = 0;      // entries of the per-tour arrays
    DevStats *d_stats = nullptr;
    int32_t cap_T = 0;
    unsigned long long *d_partials = nullptr;
    int64_t cap_partials = 0;
    BatchCtl *d_ctl = nullptr;
    int16_t *d_mask = nullptr;  // two-kernel form only: window starts [positions][S]
    int64_t cap_mask = 0;       // elements
};

void free_buffers(EvalBuffers &b)
{
    if (b.d_stage) (void)hipFree(b.d_stage);
    if (b.d_rowoff) (void)hipFree(b.d_rowoff);
    if (b.d_rowoff32) (void)hipFree(b.d_rowoff32);
    if (b.d_w) (void)hipFree(b.d_w);
    if (b.d_stats) (void)hipFree(b.d_stats);
    if (b.d_partials) (void)hipFree(b.d_partials);
    if (b.d_ctl) (void)hipFree(b.d_ctl);
    if (b.d_mask) (void)hipFree(b.d_mask);
    b = EvalBuffers();
}

// Byte offsets of the staged header for capacity capT tours and cap_n positions:
// int64 T at 0, int64 tptr[capT + 1] at 8, int32 order[capT], int32 tours[cap_n].
struct StageLayout {
    int32_t capT = 0;
    size_t off_order = 0, off_tours = 0, bytes = 0;
};

StageLayout stage_layout(int32_t capT, int64_t cap_n)
{
    StageLayout L;
    L.capT = capT;
    L.off_order = sizeof(int64_t) * (2 + (size_t)capT);
    L.off_tours = L.off_order + ((sizeof(int32_t) * (size_t)capT + 7) & ~(size_t)7);
    L.bytes = L.off_tours + sizeof(int32_t) * (size_t)cap_n;
    return L;
}

// Summary of a validated batch.
struct BatchInfo {
    int32_t T = 0, max_id = 0, maxn = 0, minn = 0;
    int64_t total_n = 0;
};

// What the kernels of one evaluation are launched with.
struct Plan {
    int form = SPLIT_FORM_LANE;
    int32_t lane_grid = 0, wave_grid = 0, maxn = 0, lane_block = 16;
    bool lane_static = false, lane_uniform = false;
    uint32_t lane_bytes = 0;
};

// The instance as the kernels see it (a graph keeps its own copy).
struct Instance {
    int32_t N = 0;
    int kind = -1;  // 0 coordinates, 1 matrix
    int32_t *d_xy = nullptr;
    int32_t *d_dist = nullptr;
    int64_t max_arc = 0;
};

void free_instance(Instance &in)
{
    if (in.d_xy) (void)hipFree(in.d_xy);
    if (in.d_dist) (void)hipFree(in.d_dist);
    in = Instance();
}

}  // namespace

struct split_ctx {
    int device = 0;
    int cus = 0;
    std::string err;
    split_tuning tuning = {SPLIT_FORM_AUTO, 0, 0, 0, 0};

    Instance inst;
    std::vector<unsigned char> seen;

    EvalBuffers buf;

    // pinned host staging
    char *h_stage[kStages] = {};
    int64_t cap_h_stage = 0;
    hipEvent_t stage_ev[kStages] = {};
    bool stage_ev_used[kStages] = {};
    int stage = 0;
    DevStats *h_stats = nullptr;
    int32_t cap_h_stats = 0;
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
    std::vector<float> ms_samples;  // per timed launch since the last reset
    const char *tname = "";

    // device address of this GPU's fixed scratch (split_eval_noalloc), looked up at creation
    unsigned char *scratch = nullptr;
};

struct split_graph {
    split_ctx *ctx = nullptr;  // for error messages and the device
    Instance inst;
    std::vector<unsigned char> seen;
    EvalBuffers buf;
    StageLayout layout;
    int32_t max_T = 0;
    int64_t max_total_n = 0;
    int64_t S = 0, ld = 0, ldc = 0;
    int32_t Q = 0;
    int order = 0;
    Plan plan;
    hipStream_t cap_stream = nullptr;
    char *h_stage[kGraphSlots] = {};
    DevStats *h_stats[kGraphSlots] = {};
    hipGraph_t graph[kGraphSlots] = {};
    hipGraphExec_t exec[kGraphSlots] = {};
    hipEvent_t done[kGraphSlots] = {};
    bool used[kGraphSlots] = {};
    int next = 0;
    int last = -1;
    int32_t last_T = 0;
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

template <class P>
bool grow(P **ptr, size_t bytes)
{
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    return hipMalloc(ptr, bytes) == hipSuccess;
}

// Device buffers for T tours with total_n positions in all, staging of stage_bytes and moment
// partials of partial_blocks blocks (exact sizes, or with room to grow). Growing waits for
// enqueued work before replacing a buffer.
split_status ensure_buffers(split_ctx *ctx, EvalBuffers &b, int32_t T, int64_t total_n,
                            int64_t stage_bytes, int64_t partial_blocks, bool exact)
{
    const int64_t pos = total_n + (int64_t)T * (1 + kRowPad);
    const bool g_pos = pos > b.cap_pos, g_stage = stage_bytes > b.cap_stage;
    const bool g_T = T > b.cap_T, g_part = partial_blocks > b.cap_partials;
    const bool g_ctl = b.d_ctl == nullptr;
    if (!g_pos && !g_stage && !g_T && !g_part && !g_ctl) return SPLIT_OK;
    HIP_TRY(ctx, hipDeviceSynchronize());
    auto room = [exact](int64_t need, int64_t floor) {
        return exact ? need : (need < floor ? floor : need + need / 4);
    };
    if (g_pos) {
        const int64_t np = room(pos, 4096);
        b.cap_pos = 0;
        if (!grow(&b.d_rowoff, sizeof(int64_t) * np) ||
            !grow(&b.d_rowoff32, sizeof(uint32_t) * np) || !grow(&b.d_w, sizeof(int32_t) * np))
            return fail(ctx, SPLIT_E_NOMEM, "device allocation for %lld tour positions failed",
                        (long long)np);
        b.cap_pos = np;
    }
    if (g_stage) {
        const int64_t nb = room(stage_bytes, 65536);
        b.cap_stage = 0;
        if (!grow(&b.d_stage, (size_t)nb))
            return fail(ctx, SPLIT_E_NOMEM, "device staging of %lld bytes failed", (long long)nb);
        b.cap_stage = nb;
    }
    if (g_T) {
        const int32_t nt = exact ? T : (T < 16 ? 16 : T);
        b.cap_T = 0;
        if (!grow(&b.d_stats, sizeof(DevStats) * nt))
            return fail(ctx, SPLIT_E_NOMEM, "allocation of %d result blocks failed", nt);
        b.cap_T = nt;
    }
    if (g_part) {
        b.cap_partials = 0;
        if (!grow(&b.d_partials, sizeof(unsigned long long) * 3 * partial_blocks))
            return fail(ctx, SPLIT_E_NOMEM, "allocation of moment partials failed");
        b.cap_partials = partial_blocks;
    }
    if (g_ctl && hipMalloc(&b.d_ctl, sizeof(BatchCtl)) != hipSuccess)
        return fail(ctx, SPLIT_E_NOMEM, "allocation of the batch counters failed");
    return SPLIT_OK;
}

// Pinned host staging of the context: kStages slots of stage_bytes and T result blocks.
split_status ensure_host(split_ctx *ctx, int64_t stage_bytes, int32_t T)
{
    if (stage_bytes > ctx->cap_h_stage) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        const int64_t nb = stage_bytes < 65536 ? 65536 : stage_bytes + stage_bytes / 4;
        ctx->cap_h_stage = 0;
        for (int k = 0; k < kStages; ++k) {
            if (ctx->h_stage[k]) (void)hipHostFree(ctx->h_stage[k]);
            ctx->h_stage[k] = nullptr;
            ctx->stage_ev_used[k] = false;
            if (hipHostMalloc((void **)&ctx->h_stage[k], (size_t)nb, 0) != hipSuccess)
                return fail(ctx, SPLIT_E_NOMEM, "pinned staging of %lld bytes failed",
                            (long long)nb);
        }
        ctx->cap_h_stage = nb;
    }
    if (T > ctx->cap_h_stats) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        const int32_t nt = T < 16 ? 16 : T;
        if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
        ctx->h_stats = nullptr;
        ctx->cap_h_stats = 0;
        if (hipHostMalloc((void **)&ctx->h_stats, sizeof(DevStats) * nt, 0) != hipSuccess)
            return fail(ctx, SPLIT_E_NOMEM, "pinned allocation of %d result blocks failed", nt);
        memset(ctx->h_stats, 0, sizeof(DevStats) * nt);
        ctx->cap_h_stats = nt;
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
        ctx->ms_samples.push_back(ms);
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

// Per-tour statistics and status of T result blocks; SPLIT_E_DEMAND names the first bad tour.
split_status report(split_ctx *ctx, const DevStats *h, int32_t T, int64_t S, split_stats *stats,
                    int32_t *tour_status)
{
    int bad = -1;
    for (int32_t t = 0; t < T; ++t) {
        if (stats) fill_stats(h[t], S, stats + t);
        if (tour_status) tour_status[t] = h[t].err_demand ? SPLIT_E_DEMAND : SPLIT_OK;
        if (h[t].err_demand && bad < 0) bad = t;
    }
    if (bad >= 0)
        return fail(ctx, SPLIT_E_DEMAND, "tour %d: a scenario has a demand q < 0 or q > Q on the "
                    "tour", bad);
    return SPLIT_OK;
}

split_status check_shape(split_ctx *ctx, const char *who, int64_t S, int64_t ld, int32_t Q,
                         int64_t ldc)
{
    if (S < 1 || S > INT32_MAX || ld < S || ldc < S)
        return fail(ctx, SPLIT_E_INVAL, "%s: need 1 <= S < 2^31, ld >= S and ldc >= S", who);
    if (Q < 1) return fail(ctx, SPLIT_E_INVAL, "%s: need Q >= 1", who);
    return SPLIT_OK;
}

// Tours against instance `in` (seen: scratch of N + 1 zeros, left zeroed), the work-item
// bound T * ceil(S / 64) < 2^31 and the int32 range of the DP.
split_status check_tours(split_ctx *ctx, const char *who, const Instance &in,
                         std::vector<unsigned char> &seen, const int32_t *tours,
                         const int64_t *tour_ptr, int32_t T, int64_t S, BatchInfo *info)
{
    if (!tours || !tour_ptr) return fail(ctx, SPLIT_E_INVAL, "%s: NULL pointer", who);
    if (T < 1) return fail(ctx, SPLIT_E_INVAL, "%s: need T >= 1", who);
    if (tour_ptr[0] != 0) return fail(ctx, SPLIT_E_INVAL, "%s: tour_ptr[0] must be 0", who);
    BatchInfo bi;
    bi.T = T;
    for (int32_t t = 0; t < T; ++t) {
        const int64_t n64 = tour_ptr[t + 1] - tour_ptr[t];
        if (n64 < 1 || n64 > in.N)
            return fail(ctx, SPLIT_E_INVAL, "%s: tour %d has length %lld (need 1..N)", who, t,
                        (long long)n64);
        const int32_t n = (int32_t)n64;
        bi.maxn = n > bi.maxn ? n : bi.maxn;
        bi.minn = (t == 0 || n < bi.minn) ? n : bi.minn;
        const int32_t *tour = tours + tour_ptr[t];
        for (int32_t k = 0; k < n; ++k) {
            const int32_t c = tour[k];
            if (c < 1 || c > in.N || seen[c]) {
                for (int32_t j = 0; j < k; ++j) seen[tour[j]] = 0;
                return fail(ctx, SPLIT_E_TOUR, "%s: tour %d position %d: id %d is out of range "
                            "or repeated", who, t, k, c);
            }
            seen[c] = 1;
            bi.max_id = c > bi.max_id ? c : bi.max_id;
        }
        for (int32_t k = 0; k < n; ++k) seen[tour[k]] = 0;
    }
    bi.total_n = tour_ptr[T];
    const int64_t nsb = (S + 63) / 64;
    if ((__int128)nsb * T >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_INVAL, "%s: T * ceil(S / 64) must be below 2^31", who);
    // |g| and |w| stay below (2n+3) * max_arc; keep them below 2^30 with a margin.
    if ((__int128)4 * ((__int128)bi.maxn + 1) * in.max_arc >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_RANGE, "%s: 4*(n+1)*max_arc = 4*%d*%lld exceeds 2^31", who,
                    bi.maxn + 1, (long long)in.max_arc);
    *info = bi;
    return SPLIT_OK;
}

// Header, work order and tours into host memory h laid out by L (T <= L.capT).
void stage_write(char *h, const StageLayout &L, const int32_t *tours, const int64_t *tour_ptr,
                 int32_t T, int order_mode)
{
    const int64_t T64 = T;
    memcpy(h, &T64, sizeof T64);
    memcpy(h + sizeof(int64_t), tour_ptr, sizeof(int64_t) * ((size_t)T + 1));
    int32_t *order = reinterpret_cast<int32_t *>(h + L.off_order);
    for (int32_t t = 0; t < T; ++t) order[t] = t;
    if (order_mode == 0) {
        // longest tours first (ties by index), so that short ones fill the tail
        std::stable_sort(order, order + T, [&](int32_t x, int32_t y) {
            return tour_ptr[x + 1] - tour_ptr[x] > tour_ptr[y + 1] - tour_ptr[y];
        });
    }
    memcpy(h + L.off_tours, tours, sizeof(int32_t) * (size_t)tour_ptr[T]);
}

// Launch configuration from the tuning. T_grid bounds T; maxn and max_id bound the tours;
// `uniform`: every tour of the launch has the same length (so has every work item).
Plan make_plan(const split_ctx *ctx, const split_tuning &tu, int64_t S, int64_t ld, int32_t Q,
               int32_t T_grid, int32_t maxn, int32_t max_id, bool uniform)
{
    Plan p;
    p.form = tu.form;
    if (p.form == SPLIT_FORM_AUTO) p.form = auto_wave(S, maxn) ? SPLIT_FORM_WAVE : SPLIT_FORM_LANE;
    // past the lane kernel's 16-bit bound every scenario would be handed to the wave kernel
    if (p.form == SPLIT_FORM_LANE && Q > kLaneMaxQ) p.form = SPLIT_FORM_WAVE;
    // the lane kernel addresses demands with 32-bit buffer offsets
    const __int128 lane_bytes = ((__int128)(max_id - 1) * ld + S) * 2;
    const bool lane_addressable = lane_bytes <= (__int128)kRowAbsent;
    p.lane_bytes = lane_addressable ? (uint32_t)lane_bytes : 0u;
    if (p.form == SPLIT_FORM_LANE && !lane_addressable) p.form = SPLIT_FORM_WAVE;
    const int64_t items = (S + 63) / 64 * T_grid;
    // The library's choice (lane_per_cu 0): over one tour with at most kLaneStaticMaxRounds
    // items per workgroup, kLaneStaticPerCu resident workgroups per compute unit taking items
    // at a fixed stride (no dispatch gap between items, no queue); otherwise one workgroup per
    // item. Measured: 8, 12 and 16 items per workgroup of one tour gain about 1%; over several
    // tours, even of one length, their items differ enough that a fixed split lost 2-3%.
    const bool lib_choice = tu.lane_per_cu <= 0;
    const int64_t sgrid = (int64_t)ctx->cus * kLaneStaticPerCu;
    const bool fixed = lib_choice && T_grid == 1 && items <= sgrid * kLaneStaticMaxRounds;
    const int64_t lg = !lib_choice ? (int64_t)ctx->cus * tu.lane_per_cu : fixed ? sgrid : items;
    p.lane_grid = (int32_t)(lg < items ? lg : items);
    p.lane_static = fixed;
    p.lane_uniform = uniform;
    p.lane_block = tu.lane_block == 8 ? 8 : 16;
    p.wave_grid = tu.wave_grid > 0 ? tu.wave_grid : 65536;
    p.maxn = maxn;
    return p;
}

// The kernels of one evaluation on `stream`, reading the header already staged in b.d_stage
// (laid out by L): prep, the Split DP (lane kernel and its fallback, or the wave kernel),
// moments. The dominant kernel is timed when ctx->timing and `timed` are set.
split_status enqueue_kernels(split_ctx *ctx, const Instance &in, const EvalBuffers &b,
                             const StageLayout &L, const Plan &p, const int16_t *demand,
                             int64_t S, int64_t ld, int32_t Q, int32_t *cost, int64_t ldc,
                             hipStream_t stream, bool timed)
{
    TourDev td;
    td.nt = reinterpret_cast<const int64_t *>(b.d_stage);
    td.tptr = td.nt + 1;
    td.order = reinterpret_cast<const int32_t *>(b.d_stage + L.off_order);
    td.tours = reinterpret_cast<const int32_t *>(b.d_stage + L.off_tours);
    td.T_grid = L.capT;
    td.rowoff = b.d_rowoff;
    td.rowoff32 = b.d_rowoff32;
    td.w = b.d_w;

    PrepArgs pa;
    pa.tour = td;
    pa.N = in.N;
    pa.kind = in.kind;
    pa.xy = in.d_xy;
    pa.dist = in.d_dist;
    pa.ld = ld;
    pa.stats = b.d_stats;
    pa.ctl = b.d_ctl;
    HIP_TRY(ctx, launch_prep(pa, stream));

    EvalArgs ea;
    ea.demand = reinterpret_cast<const uint16_t *>(demand);
    ea.ld = ld;
    ea.S = S;
    ea.Q = Q;
    ea.tour = td;
    ea.cost = cost;
    ea.ldc = ldc;
    ea.stats = b.d_stats;
    ea.ctl = b.d_ctl;
    ea.lane_bytes = p.lane_bytes;
    ea.lane_grid = p.lane_grid;
    ea.lane_static = p.lane_static ? 1 : 0;
    ea.lane_uniform = p.lane_uniform ? 1 : 0;
    ea.lane_block = p.lane_block;
    ea.wave_grid = p.wave_grid;
    ea.maxn = p.maxn;

    hipEvent_t stop = nullptr;
    if (timed) {
        split_status st = timing_begin(ctx, stream, &stop);
        if (st != SPLIT_OK) return st;
    }
    if (p.form == SPLIT_FORM_WAVE) {
        ctx->tname = wave_kernel_name();
        HIP_TRY(ctx, launch_wave_all(ea, stream));
        if (stop) HIP_TRY(ctx, hipEventRecord(stop, stream));
    } else if (p.form == SPLIT_FORM_MASK) {
        ctx->tname = mask_kernel_name();
        HIP_TRY(ctx, launch_mask(ea, b.d_mask, S, stream));
        HIP_TRY(ctx, launch_masked_dp(ea, b.d_mask, S, stream));
        if (stop) HIP_TRY(ctx, hipEventRecord(stop, stream));
        HIP_TRY(ctx, launch_wave_fallback(ea, stream));
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
    ma.nt = td.nt;
    ma.T_grid = L.capT;
    ma.partials = b.d_partials;
    ma.nblocks = moment_blocks(S);
    ma.stats = b.d_stats;
    HIP_TRY(ctx, launch_moments(ma, stream));
    return SPLIT_OK;
}

// The common path of split_eval and split_eval_batch on the context's own buffers.
split_status eval_batch(split_ctx *ctx, const char *who, const int32_t *tours,
                        const int64_t *tour_ptr, int32_t T, const int16_t *demand, int64_t S,
                        int64_t ld, int32_t Q, int32_t *cost, int64_t ldc, hipStream_t stream)
{
    if (ctx->inst.kind < 0) return fail(ctx, SPLIT_E_INVAL, "%s: no instance set", who);
    if (!demand || !cost) return fail(ctx, SPLIT_E_INVAL, "%s: NULL pointer", who);
    split_status st = check_shape(ctx, who, S, ld, Q, ldc);
    if (st != SPLIT_OK) return st;
    BatchInfo bi;
    st = check_tours(ctx, who, ctx->inst, ctx->seen, tours, tour_ptr, T, S, &bi);
    if (st != SPLIT_OK) return st;

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    const StageLayout L = stage_layout(T, bi.total_n);
    const int32_t nblk = moment_blocks(S);
    st = ensure_buffers(ctx, ctx->buf, T, bi.total_n, (int64_t)L.bytes, (int64_t)nblk * T, false);
    if (st != SPLIT_OK) return st;
    st = ensure_host(ctx, (int64_t)L.bytes, T);
    if (st != SPLIT_OK) return st;

    // Upload through a pinned slot, reused only after its previous copy completed.
    const int slot = ctx->stage;
    ctx->stage = (ctx->stage + 1) % kStages;
    if (ctx->stage_ev_used[slot]) HIP_TRY(ctx, hipEventSynchronize(ctx->stage_ev[slot]));
    stage_write(ctx->h_stage[slot], L, tours, tour_ptr, T, ctx->tuning.order);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->buf.d_stage, ctx->h_stage[slot], L.bytes,
                                hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipEventRecord(ctx->stage_ev[slot], stream));
    ctx->stage_ev_used[slot] = true;

    const Plan p = make_plan(ctx, ctx->tuning, S, ld, Q, T, bi.maxn, bi.max_id,
                             bi.minn == bi.maxn);
    if (p.form == SPLIT_FORM_MASK && (__int128)ctx->buf.cap_pos * S > ctx->buf.cap_mask) {
        // one int16 window start per (position row, scenario)
        HIP_TRY(ctx, hipDeviceSynchronize());
        if (ctx->buf.d_mask) (void)hipFree(ctx->buf.d_mask);
        ctx->buf.d_mask = nullptr;
        ctx->buf.cap_mask = 0;
        const int64_t elems = ctx->buf.cap_pos * S;
        if (hipMalloc(&ctx->buf.d_mask, sizeof(int16_t) * (size_t)elems) != hipSuccess)
            return fail(ctx, SPLIT_E_NOMEM, "%s: the two-kernel form's %lld-byte mask matrix "
                        "could not be allocated", who, (long long)(2 * elems));
        ctx->buf.cap_mask = elems;
    }
    st = enqueue_kernels(ctx, ctx->inst, ctx->buf, L, p, demand, S, ld, Q, cost, ldc, stream, true);
    if (st != SPLIT_OK) return st;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_stats, ctx->buf.d_stats, sizeof(DevStats) * (size_t)T,
                                hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipEventRecord(ctx->stats_ev, stream));
    ctx->have_call = true;
    ctx->last_S = S;
    ctx->last_T = T;
    return SPLIT_OK;
}

split_status check_tuning(split_ctx *ctx, const split_tuning &t)
{
    if (t.form != SPLIT_FORM_AUTO && t.form != SPLIT_FORM_LANE && t.form != SPLIT_FORM_WAVE &&
        t.form != SPLIT_FORM_MASK)
        return fail(ctx, SPLIT_E_INVAL, "tuning: unknown form %d", t.form);
    if (t.lane_per_cu < 0 || t.lane_per_cu > kMaxLanePerCu)
        return fail(ctx, SPLIT_E_INVAL, "tuning: lane_per_cu must be in 0..%d", kMaxLanePerCu);
    if (t.order != 0 && t.order != 1)
        return fail(ctx, SPLIT_E_INVAL, "tuning: order must be 0 or 1");
    if (t.wave_grid < 0) return fail(ctx, SPLIT_E_INVAL, "tuning: wave_grid must be >= 0");
    if (t.lane_block != 0 && t.lane_block != 8 && t.lane_block != 16)
        return fail(ctx, SPLIT_E_INVAL, "tuning: lane_block must be 0, 8 or 16");
    return SPLIT_OK;
}

}  // namespace

namespace splitgpu {

int ctx_device(const split_ctx *ctx) { return ctx->device; }

bool ctx_instance(const split_ctx *ctx, int32_t *N, int *kind, const int32_t **xy,
                  const int32_t **dist, int64_t *max_arc)
{
    if (ctx->inst.kind < 0) return false;
    *N = ctx->inst.N;
    *kind = ctx->inst.kind;
    *xy = ctx->inst.d_xy;
    *dist = ctx->inst.d_dist;
    *max_arc = ctx->inst.max_arc;
    return true;
}

split_status ctx_fail(split_ctx *ctx, split_status st, const char *fmt, ...)
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

}  // namespace splitgpu

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
        hipEventCreateWithFlags(&ctx->stats_ev, hipEventDisableTiming) != hipSuccess) {
        split_ctx_destroy(ctx);
        return SPLIT_E_NOMEM;
    }
    ctx->cus = prop.multiProcessorCount;
    void *scr = nullptr;
    if (scratch_address(hip_device, &scr) != hipSuccess) {
        split_ctx_destroy(ctx);
        return SPLIT_E_HIP;
    }
    ctx->scratch = static_cast<unsigned char *>(scr);
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
        free_instance(ctx->inst);
        free_buffers(ctx->buf);
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
    free_instance(ctx->inst);
    HIP_TRY(ctx, hipMalloc(&ctx->inst.d_xy, sizeof(int32_t) * 2 * ((size_t)N + 1)));
    HIP_TRY(ctx, hipMemcpy(ctx->inst.d_xy, xy, sizeof(int32_t) * 2 * ((size_t)N + 1),
                           hipMemcpyHostToDevice));
    const double dx = (double)(hi[0] - lo[0]), dy = (double)(hi[1] - lo[1]);
    ctx->inst.max_arc = (int64_t)ceil(sqrt(dx * dx + dy * dy)) + 1;  // bound on any rounded distance
    ctx->inst.N = N;
    ctx->inst.kind = 0;
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
    free_instance(ctx->inst);
    HIP_TRY(ctx, hipMalloc(&ctx->inst.d_dist, sizeof(int32_t) * V * V));
    HIP_TRY(ctx, hipMemcpy(ctx->inst.d_dist, d, sizeof(int32_t) * V * V, hipMemcpyHostToDevice));
    ctx->inst.max_arc = mx;
    ctx->inst.N = N;
    ctx->inst.kind = 1;
    ctx->seen.assign(V, 0);
    return SPLIT_OK;
}

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

// The largest call (a tour of SPLIT_MAX_N positions, 1024 moment blocks) fits the scratch.
static_assert(((32 + 4 * (size_t)SPLIT_MAX_N + 255) & ~(size_t)255) +
                  ((8 * ((size_t)SPLIT_MAX_N + 1 + kRowPad) + 255) & ~(size_t)255) +
                  2 * ((4 * ((size_t)SPLIT_MAX_N + 1 + kRowPad) + 255) & ~(size_t)255) +
                  2 * 256 + 24 * 1024 <= kScratchBytes,
              "split_eval_noalloc: the scratch does not hold a maximal tour");

split_status split_eval_noalloc(split_ctx *ctx, const int32_t *tour, int32_t n,
                                const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                                int32_t *cost, split_stats *stats, void *hip_stream)
{
    if (!ctx) return SPLIT_E_INVAL;
    const char *who = "split_eval_noalloc";
    if (ctx->inst.kind < 0) return fail(ctx, SPLIT_E_INVAL, "%s: no instance set", who);
    if (!demand || !cost) return fail(ctx, SPLIT_E_INVAL, "%s: NULL pointer", who);
    split_status st = check_shape(ctx, who, S, ld, Q, S);
    if (st != SPLIT_OK) return st;
    const int64_t tour_ptr[2] = {0, n};
    BatchInfo bi;
    st = check_tours(ctx, who, ctx->inst, ctx->seen, tour, tour_ptr, 1, S, &bi);
    if (st != SPLIT_OK) return st;
    split_tuning tu = ctx->tuning;
    if (tu.form == SPLIT_FORM_MASK)
        return fail(ctx, SPLIT_E_INVAL, "%s: the two-kernel form needs a mask matrix in device "
                    "memory and is not available without allocation", who);

    // Carve the call's device buffers from the scratch, each 256-byte aligned.
    const StageLayout L = stage_layout(1, n);
    const int64_t pos = (int64_t)n + 1 + kRowPad;
    const int32_t nblk = moment_blocks(S);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_stage = 0;
    const size_t o_rowoff = o_stage + up(L.bytes);
    const size_t o_rowoff32 = o_rowoff + up(sizeof(int64_t) * (size_t)pos);
    const size_t o_w = o_rowoff32 + up(sizeof(uint32_t) * (size_t)pos);
    const size_t o_stats = o_w + up(sizeof(int32_t) * (size_t)pos);
    const size_t o_ctl = o_stats + up(sizeof(DevStats));
    const size_t o_part = o_ctl + up(sizeof(BatchCtl));
    const size_t need = o_part + up(sizeof(unsigned long long) * 3 * (size_t)nblk);
    if (need > kScratchBytes)
        return fail(ctx, SPLIT_E_INVAL, "%s: a tour of %d positions needs %zu bytes of device "
                    "scratch, above the fixed %zu", who, n, need, kScratchBytes);

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    EvalBuffers b;  // views of the scratch; nothing here is owned or freed
    b.d_stage = reinterpret_cast<char *>(ctx->scratch + o_stage);
    b.cap_stage = (int64_t)L.bytes;
    b.d_rowoff = reinterpret_cast<int64_t *>(ctx->scratch + o_rowoff);
    b.d_rowoff32 = reinterpret_cast<uint32_t *>(ctx->scratch + o_rowoff32);
    b.d_w = reinterpret_cast<int32_t *>(ctx->scratch + o_w);
    b.cap_pos = pos;
    b.d_stats = reinterpret_cast<DevStats *>(ctx->scratch + o_stats);
    b.cap_T = 1;
    b.d_ctl = reinterpret_cast<BatchCtl *>(ctx->scratch + o_ctl);
    b.d_partials = reinterpret_cast<unsigned long long *>(ctx->scratch + o_part);
    b.cap_partials = nblk;

    // The staged header of a batch of one: T, tptr, order, then the tour itself, copied from
    // pageable host memory (the runtime stages it before the call returns).
    const hipStream_t stream = (hipStream_t)hip_stream;
    const int64_t head[3] = {1, 0, n};
    const int32_t order0 = 0;
    HIP_TRY(ctx, hipMemcpyAsync(b.d_stage, head, sizeof head, hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.d_stage + L.off_order, &order0, sizeof order0,
                                hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.d_stage + L.off_tours, tour, sizeof(int32_t) * (size_t)n,
                                hipMemcpyHostToDevice, stream));
    const Plan p = make_plan(ctx, tu, S, ld, Q, 1, bi.maxn, bi.max_id, true);
    // the prep kernel zeroes the result block and the counters of every call
    st = enqueue_kernels(ctx, ctx->inst, b, L, p, demand, S, ld, Q, cost, S, stream, false);
    if (st != SPLIT_OK) return st;
    if (!stats) return SPLIT_OK;
    DevStats d;
    HIP_TRY(ctx, hipMemcpyAsync(&d, b.d_stats, sizeof d, hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    fill_stats(d, S, stats);
    if (d.err_demand)
        return fail(ctx, SPLIT_E_DEMAND, "%s: a scenario has a demand q < 0 or q > Q on the tour",
                    who);
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
    return report(ctx, ctx->h_stats, ctx->last_T, ctx->last_S, stats, tour_status);
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
    if (form != SPLIT_FORM_AUTO && form != SPLIT_FORM_LANE && form != SPLIT_FORM_WAVE &&
        form != SPLIT_FORM_MASK)
        return fail(ctx, SPLIT_E_INVAL, "split_set_form: unknown form %d", form);
    ctx->tuning.form = form;
    return SPLIT_OK;
}

split_status split_tuning_set(split_ctx *ctx, const split_tuning *tuning)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!tuning) return fail(ctx, SPLIT_E_INVAL, "split_tuning_set: NULL tuning");
    split_status st = check_tuning(ctx, *tuning);
    if (st != SPLIT_OK) return st;
    ctx->tuning = *tuning;
    return SPLIT_OK;
}

split_status split_tuning_get(split_ctx *ctx, split_tuning *tuning)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!tuning) return fail(ctx, SPLIT_E_INVAL, "split_tuning_get: NULL tuning");
    *tuning = ctx->tuning;
    return SPLIT_OK;
}

split_status split_autotune(split_ctx *ctx, const int32_t *tours, const int64_t *tour_ptr,
                            int32_t T, const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                            int32_t *cost, int64_t ldc, int32_t reps, void *hip_stream,
                            split_tuning *best, double *best_ms)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (reps < 1 || reps > 1000)
        return fail(ctx, SPLIT_E_INVAL, "split_autotune: need 1 <= reps <= 1000");
    if (ctx->inst.kind < 0) return fail(ctx, SPLIT_E_INVAL, "split_autotune: no instance set");
    if (!demand || !cost) return fail(ctx, SPLIT_E_INVAL, "split_autotune: NULL pointer");
    split_status st = check_shape(ctx, "split_autotune", S, ld, Q, ldc);
    if (st != SPLIT_OK) return st;
    BatchInfo bi;
    st = check_tours(ctx, "split_autotune", ctx->inst, ctx->seen, tours, tour_ptr, T, S, &bi);
    if (st != SPLIT_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    hipStream_t stream = (hipStream_t)hip_stream;

    const split_tuning saved = ctx->tuning;
    const bool saved_timing = ctx->timing;
    ctx->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto finish = [&](split_status s) {
        ctx->timing = saved_timing;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s != SPLIT_OK) ctx->tuning = saved;
        return s;
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return finish(fail(ctx, SPLIT_E_HIP, "split_autotune: hipEventCreate failed"));

    // mean milliseconds of one whole evaluation (upload, kernels, statistics) under tuning c,
    // on the first s_eval scenarios
    auto measure = [&](const split_tuning &c, int64_t s_eval, double *ms) -> split_status {
        ctx->tuning = c;
        split_status s = eval_batch(ctx, "split_autotune", tours, tour_ptr, T, demand, s_eval, ld,
                                    Q, cost, ldc, stream);  // warm-up
        if (s != SPLIT_OK) return s;
        s = split_batch_stats_get(ctx, nullptr, nullptr);
        if (s != SPLIT_OK) return s;
        if (hipEventRecord(e0, stream) != hipSuccess)
            return fail(ctx, SPLIT_E_HIP, "split_autotune: hipEventRecord failed");
        for (int r = 0; r < reps; ++r) {
            s = eval_batch(ctx, "split_autotune", tours, tour_ptr, T, demand, s_eval, ld, Q, cost,
                           ldc, stream);
            if (s != SPLIT_OK) return s;
        }
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fail(ctx, SPLIT_E_HIP, "split_autotune: timing events failed");
        float el = 0.f;
        if (hipEventElapsedTime(&el, e0, e1) != hipSuccess)
            return fail(ctx, SPLIT_E_HIP, "split_autotune: hipEventElapsedTime failed");
        *ms = (double)el / reps;
        return split_batch_stats_get(ctx, nullptr, nullptr);
    };

    // scenarios left to the wave kernel, over the first s_eval scenarios, under tuning c
    std::vector<split_stats> fb_stats((size_t)T);
    auto fallbacks = [&](const split_tuning &c, int64_t s_eval, int64_t *n) -> split_status {
        ctx->tuning = c;
        split_status s = eval_batch(ctx, "split_autotune", tours, tour_ptr, T, demand, s_eval, ld,
                                    Q, cost, ldc, stream);
        if (s != SPLIT_OK) return s;
        s = split_batch_stats_get(ctx, fb_stats.data(), nullptr);
        if (s != SPLIT_OK) return s;
        *n = 0;
        for (const split_stats &x : fb_stats) *n += x.n_fallback;
        return SPLIT_OK;
    };

    split_tuning win = saved;
    double win_ms = 1e300;
    const Plan lane_probe = make_plan(ctx, split_tuning{SPLIT_FORM_LANE, 0, 0, 0, 0}, S, ld, Q,
                                      T, bi.maxn, bi.max_id, bi.minn == bi.maxn);
    if (lane_probe.form == SPLIT_FORM_LANE) {
        // the block length first (it follows the window lengths, so the demand law), then the
        // grid and the order with that block length. 8-state blocks hand windows longer than
        // about 24 positions to the wave kernel, which costs far more than any block saves: a
        // probe on the first scenarios drops them when they leave more scenarios there.
        const int64_t s_fb = S < 4096 ? S : 4096;
        int64_t fb16 = 0, fb8 = 0;
        st = fallbacks(split_tuning{SPLIT_FORM_LANE, 0, 0, 0, 16}, s_fb, &fb16);
        if (st != SPLIT_OK) return finish(st);
        st = fallbacks(split_tuning{SPLIT_FORM_LANE, 0, 0, 0, 8}, s_fb, &fb8);
        if (st != SPLIT_OK) return finish(st);
        int32_t block = 16;
        for (int32_t lb : {16, 8}) {
            if (lb == 8 && fb8 > fb16) continue;
            const split_tuning c = {SPLIT_FORM_LANE, 0, 0, 0, lb};
            double ms = 0.0;
            st = measure(c, S, &ms);
            if (st != SPLIT_OK) return finish(st);
            if (ms < win_ms) {
                win_ms = ms;
                win = c;
                block = lb;
            }
        }
        const int32_t per_cu[] = {0, 8, 4, 2};
        for (int32_t pc : per_cu)
            for (int32_t order = 0; order < 2; ++order) {
                if (T == 1 && order == 1) continue;  // one tour: the order is moot
                if (pc == 0 && order == 0) continue;  // timed above
                const split_tuning c = {SPLIT_FORM_LANE, pc, order, 0, block};
                double ms = 0.0;
                st = measure(c, S, &ms);
                if (st != SPLIT_OK) return finish(st);
                if (ms < win_ms) {
                    win_ms = ms;
                    win = c;
                }
            }
    }
    // The wave form costs about S times one scenario's evaluation: try it in full only when a
    // run on at most 256 scenarios, scaled to S, is within 1.5x of the best so far.
    const int64_t s_probe = S < 256 ? S : 256;
    double probe_ms = 0.0;
    st = measure(split_tuning{SPLIT_FORM_WAVE, 0, 0, 0, 0}, s_probe, &probe_ms);
    if (st != SPLIT_OK) return finish(st);
    if (probe_ms * ((double)S / (double)s_probe) < 1.5 * win_ms) {
        const int32_t grids[] = {0, ctx->cus * 8};
        for (int32_t wg : grids) {
            const split_tuning c = {SPLIT_FORM_WAVE, 0, 0, wg, 0};
            double ms = 0.0;
            st = measure(c, S, &ms);
            if (st != SPLIT_OK) return finish(st);
            if (ms < win_ms) {
                win_ms = ms;
                win = c;
            }
        }
    }
    // leave the context's latest evaluation the full one under the chosen tuning
    ctx->tuning = win;
    st = eval_batch(ctx, "split_autotune", tours, tour_ptr, T, demand, S, ld, Q, cost, ldc, stream);
    if (st != SPLIT_OK) return finish(st);
    st = split_batch_stats_get(ctx, nullptr, nullptr);
    if (st != SPLIT_OK) return finish(st);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return finish(SPLIT_OK);
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
    ctx->ms_samples.clear();
    return st;
}

split_status split_timing_samples(split_ctx *ctx, float *ms, int64_t cap, int64_t *count)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (cap < 0 || (cap > 0 && !ms))
        return fail(ctx, SPLIT_E_INVAL, "split_timing_samples: need cap >= 0 and ms for cap > 0");
    DeviceGuard g(ctx->device);
    split_status st = collect_timing(ctx);
    if (st != SPLIT_OK) return st;
    const int64_t n = (int64_t)ctx->ms_samples.size();
    for (int64_t k = 0; k < n && k < cap; ++k) ms[k] = ctx->ms_samples[(size_t)k];
    if (count) *count = n;
    return SPLIT_OK;
}

// ------------------------------------------------------------------------- graphs

void split_graph_destroy(split_graph *gr)
{
    if (!gr) return;
    {
        DeviceGuard g(gr->ctx->device);
        for (int k = 0; k < kGraphSlots; ++k)
            if (gr->used[k]) (void)hipEventSynchronize(gr->done[k]);
        for (int k = 0; k < kGraphSlots; ++k) {
            if (gr->exec[k]) (void)hipGraphExecDestroy(gr->exec[k]);
            if (gr->graph[k]) (void)hipGraphDestroy(gr->graph[k]);
            if (gr->done[k]) (void)hipEventDestroy(gr->done[k]);
            if (gr->h_stage[k]) (void)hipHostFree(gr->h_stage[k]);
            if (gr->h_stats[k]) (void)hipHostFree(gr->h_stats[k]);
        }
        if (gr->cap_stream) (void)hipStreamDestroy(gr->cap_stream);
        free_buffers(gr->buf);
        free_instance(gr->inst);
    }
    delete gr;
}

split_status split_graph_create(split_ctx *ctx, int32_t max_T, int64_t max_total_n,
                                const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                                int32_t *cost, int64_t ldc, split_graph **out)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!out) return fail(ctx, SPLIT_E_INVAL, "split_graph_create: NULL out");
    *out = nullptr;
    if (ctx->inst.kind < 0) return fail(ctx, SPLIT_E_INVAL, "split_graph_create: no instance set");
    if (!demand || !cost) return fail(ctx, SPLIT_E_INVAL, "split_graph_create: NULL pointer");
    split_status st = check_shape(ctx, "split_graph_create", S, ld, Q, ldc);
    if (st != SPLIT_OK) return st;
    if (max_T < 1 || max_total_n < max_T || max_total_n > (int64_t)max_T * ctx->inst.N)
        return fail(ctx, SPLIT_E_INVAL, "split_graph_create: need 1 <= max_T <= max_total_n <= "
                    "max_T * N");
    if ((__int128)((S + 63) / 64) * max_T >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_INVAL, "split_graph_create: max_T * ceil(S / 64) must be below "
                    "2^31");
    const int32_t N = ctx->inst.N;
    if ((__int128)4 * ((__int128)N + 1) * ctx->inst.max_arc >= ((__int128)1 << 31))
        return fail(ctx, SPLIT_E_RANGE, "split_graph_create: 4*(N+1)*max_arc exceeds 2^31");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");

    split_graph *gr = new (std::nothrow) split_graph();
    if (!gr) return fail(ctx, SPLIT_E_NOMEM, "split_graph_create: out of host memory");
    gr->ctx = ctx;
    bool capturing = false;
    auto bail = [&](split_status s) {
        if (capturing) {
            hipGraph_t dropped = nullptr;
            (void)hipStreamEndCapture(gr->cap_stream, &dropped);
            if (dropped) (void)hipGraphDestroy(dropped);
        }
        split_graph_destroy(gr);
        return s;
    };
    // the graph's own copy of the instance: later changes to the context's do not reach it
    gr->inst.N = N;
    gr->inst.kind = ctx->inst.kind;
    gr->inst.max_arc = ctx->inst.max_arc;
    const size_t V = (size_t)N + 1;
    if (ctx->inst.kind == 0) {
        if (hipMalloc(&gr->inst.d_xy, sizeof(int32_t) * 2 * V) != hipSuccess ||
            hipMemcpy(gr->inst.d_xy, ctx->inst.d_xy, sizeof(int32_t) * 2 * V,
                      hipMemcpyDeviceToDevice) != hipSuccess)
            return bail(fail(ctx, SPLIT_E_NOMEM, "split_graph_create: instance copy failed"));
    } else {
        if (hipMalloc(&gr->inst.d_dist, sizeof(int32_t) * V * V) != hipSuccess ||
            hipMemcpy(gr->inst.d_dist, ctx->inst.d_dist, sizeof(int32_t) * V * V,
                      hipMemcpyDeviceToDevice) != hipSuccess)
            return bail(fail(ctx, SPLIT_E_NOMEM, "split_graph_create: instance copy failed"));
    }
    gr->seen.assign(V, 0);
    gr->max_T = max_T;
    gr->max_total_n = max_total_n;
    gr->S = S;
    gr->ld = ld;
    gr->ldc = ldc;
    gr->Q = Q;
    gr->order = ctx->tuning.order;
    gr->layout = stage_layout(max_T, max_total_n);
    const int32_t nblk = moment_blocks(S);
    st = ensure_buffers(ctx, gr->buf, max_T, max_total_n, (int64_t)gr->layout.bytes,
                        (int64_t)nblk * max_T, true);
    if (st != SPLIT_OK) return bail(st);
    // any tour of the instance: lengths up to N, ids up to N
    // the tours of a replay are known only then: a fixed item stride only for one tour
    gr->plan = make_plan(ctx, ctx->tuning, S, ld, Q, max_T, N, N, max_T == 1);
    if (gr->plan.form == SPLIT_FORM_MASK)
        return bail(fail(ctx, SPLIT_E_INVAL, "split_graph_create: the two-kernel form is an "
                         "ablation and is not captured"));
    if (hipStreamCreateWithFlags(&gr->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        gr->cap_stream = nullptr;
        return bail(fail(ctx, SPLIT_E_HIP, "split_graph_create: hipStreamCreate failed"));
    }
    for (int k = 0; k < kGraphSlots; ++k) {
        if (hipHostMalloc((void **)&gr->h_stage[k], gr->layout.bytes, 0) != hipSuccess ||
            hipHostMalloc((void **)&gr->h_stats[k], sizeof(DevStats) * (size_t)max_T, 0) !=
                hipSuccess)
            return bail(fail(ctx, SPLIT_E_NOMEM, "split_graph_create: pinned allocation failed"));
        memset(gr->h_stage[k], 0, gr->layout.bytes);
        if (hipEventCreateWithFlags(&gr->done[k], hipEventDisableTiming) != hipSuccess)
            return bail(fail(ctx, SPLIT_E_HIP, "split_graph_create: hipEventCreate failed"));
    }
    // one graph per host slot: upload of the slot's header, the kernels, the statistics copy
    for (int k = 0; k < kGraphSlots; ++k) {
        if (hipStreamBeginCapture(gr->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return bail(fail(ctx, SPLIT_E_HIP, "split_graph_create: hipStreamBeginCapture failed"));
        capturing = true;
        if (hipMemcpyAsync(gr->buf.d_stage, gr->h_stage[k], gr->layout.bytes,
                           hipMemcpyHostToDevice, gr->cap_stream) != hipSuccess)
            return bail(fail(ctx, SPLIT_E_HIP, "split_graph_create: capture of the upload failed"));
        st = enqueue_kernels(ctx, gr->inst, gr->buf, gr->layout, gr->plan, demand, S, ld, Q, cost,
                             ldc, gr->cap_stream, false);
        if (st != SPLIT_OK) return bail(st);
        if (hipMemcpyAsync(gr->h_stats[k], gr->buf.d_stats, sizeof(DevStats) * (size_t)max_T,
                           hipMemcpyDeviceToHost, gr->cap_stream) != hipSuccess)
            return bail(fail(ctx, SPLIT_E_HIP, "split_graph_create: capture of the copy failed"));
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(gr->cap_stream, &graph);
        capturing = false;
        gr->graph[k] = graph;
        if (e != hipSuccess || !graph)
            return bail(hip_fail(ctx, e, "split_graph_create: hipStreamEndCapture"));
        if (hipGraphInstantiate(&gr->exec[k], graph, nullptr, nullptr, 0) != hipSuccess) {
            gr->exec[k] = nullptr;
            return bail(fail(ctx, SPLIT_E_HIP, "split_graph_create: hipGraphInstantiate failed"));
        }
    }
    *out = gr;
    return SPLIT_OK;
}

split_status split_graph_launch(split_graph *gr, const int32_t *tours, const int64_t *tour_ptr,
                                int32_t T, void *hip_stream)
{
    if (!gr) return SPLIT_E_INVAL;
    split_ctx *ctx = gr->ctx;
    if (T > gr->max_T)
        return fail(ctx, SPLIT_E_INVAL, "split_graph_launch: T = %d exceeds the graph's %d", T,
                    gr->max_T);
    BatchInfo bi;
    split_status st = check_tours(ctx, "split_graph_launch", gr->inst, gr->seen, tours, tour_ptr,
                                  T, gr->S, &bi);
    if (st != SPLIT_OK) return st;
    if (bi.total_n > gr->max_total_n)
        return fail(ctx, SPLIT_E_INVAL, "split_graph_launch: %lld positions exceed the graph's "
                    "%lld", (long long)bi.total_n, (long long)gr->max_total_n);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, SPLIT_E_HIP, "hipSetDevice failed");
    const int k = gr->next;
    if (gr->used[k]) HIP_TRY(ctx, hipEventSynchronize(gr->done[k]));
    stage_write(gr->h_stage[k], gr->layout, tours, tour_ptr, T, gr->order);
    hipStream_t stream = (hipStream_t)hip_stream;
    HIP_TRY(ctx, hipGraphLaunch(gr->exec[k], stream));
    HIP_TRY(ctx, hipEventRecord(gr->done[k], stream));
    gr->used[k] = true;
    gr->last = k;
    gr->last_T = T;
    gr->next = (k + 1) % kGraphSlots;
    return SPLIT_OK;
}

split_status split_graph_stats(split_graph *gr, split_stats *stats, int32_t *tour_status)
{
    if (!gr) return SPLIT_E_INVAL;
    split_ctx *ctx = gr->ctx;
    if (gr->last < 0) return fail(ctx, SPLIT_E_INVAL, "split_graph_stats: no launch yet");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, hipEventSynchronize(gr->done[gr->last]));
    return report(ctx, gr->h_stats[gr->last], gr->last_T, gr->S, stats, tour_status);
}

}  // extern "C"
