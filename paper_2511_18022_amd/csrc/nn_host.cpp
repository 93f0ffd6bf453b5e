// C-ABI host layer of the tour-encoder surrogate (include/split_nn.h): parameters and Adam
// state, activation buffers, the forward and backward launch sequences, the training loop,
// checkpoints, top-k selection and screening with exact re-evaluation of the shortlist.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/split_nn.h"
#include "nn_internal.h"
#include "split_internal.h"

using namespace splitgpu;

static_assert(SPLIT_NN_PARAMS == kNnParams, "header and kernels disagree on the parameter count");

namespace {

constexpr int32_t kPredChunk = 1024;   // tours per forward pass when predicting many tours
constexpr int32_t kWgradChunk = 1024;  // padded rows per weight-gradient partial sum
constexpr int32_t kExactChunk = 256;   // shortlisted tours per exact batch evaluation
const char kMagic[8] = {'S', 'P', 'L', 'I', 'T', 'N', 'N', '1'};

uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

// Scratch of one top-k selection.
struct TopkScratch {
    NnSelect *sel = nullptr;
    unsigned long long *hist = nullptr, *base = nullptr;
    unsigned int *cnt = nullptr;
    int64_t cap_blocks = 0;
};

void free_topk(TopkScratch &k)
{
    if (k.sel) (void)hipFree(k.sel);
    if (k.hist) (void)hipFree(k.hist);
    if (k.base) (void)hipFree(k.base);
    if (k.cnt) (void)hipFree(k.cnt);
    k = TopkScratch();
}

}  // namespace

struct split_nn {
    split_ctx *ctx = nullptr;
    int device = 0;
    double L = 1.0, shift = 0.0, scale = 1.0;
    int64_t step = 0;
    float *P = nullptr, *m = nullptr, *v = nullptr, *G = nullptr;
    NnWeights w = {};
    double *musd = nullptr;
    int32_t musd_N = 0, Q = 0;
    bool have_scen = false;
    // activations [T][n + 4][C]
    uint16_t *X = nullptr, *H[4] = {}, *dP[2] = {};
    int64_t cap_rows = 0;
    int32_t zero_n = -1;  // the tour length the padding rows were cleared for
    float *z = nullptr, *a = nullptr, *y = nullptr, *da = nullptr, *dz = nullptr, *dy = nullptr;
    float *lterms = nullptr, *lout = nullptr;
    int32_t cap_T = 0;
    float *partW = nullptr, *partB = nullptr;
    int64_t cap_chunks = 0;
    float *zpart = nullptr;  // prediction: per-tile channel sums [T][tiles][128]
    int64_t cap_zpart = 0;
    uint16_t *Xp = nullptr;  // prediction: packed features [T][n][8]
    int64_t cap_xp = 0;      // positions
    int32_t *err = nullptr;
    int32_t *h_err = nullptr;  // pinned
    // training batches
    int32_t *btours = nullptr, *perm = nullptr;
    float *blabels = nullptr, *losshist = nullptr;
    int64_t cap_btours = 0, cap_perm = 0, cap_losshist = 0;
    int32_t cap_blab = 0;
    // screening
    TopkScratch tk;
    float *pred = nullptr;
    int64_t cap_pred = 0;
    int32_t *sidx = nullptr, *stours = nullptr;
    int64_t cap_sidx = 0, cap_stours = 0;
    int32_t *ecost = nullptr;
    int64_t cap_ecost = 0;
    // timing of the fused prediction kernel
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tpairs;
    size_t tpairs_used = 0;
    double ms_acc = 0.0;
    int64_t launches = 0;
};

namespace {

#define NN_TRY(nn, expr)                                                               \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ctx_fail((nn)->ctx, SPLIT_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Guard {
    int prev = -1;
    bool ok = false;
    explicit Guard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~Guard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class P>
bool realloc_dev(P **p, size_t bytes)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    return hipMalloc(p, bytes) == hipSuccess;
}

bool instance_of(split_nn *nn, NnInstance *in, int64_t *max_arc)
{
    int32_t N = 0;
    int kind = 0;
    const int32_t *xy = nullptr, *dist = nullptr;
    if (!ctx_instance(nn->ctx, &N, &kind, &xy, &dist, max_arc)) return false;
    in->N = N;
    in->kind = kind;
    in->xy = xy;
    in->dist = dist;
    return true;
}

// The per-tour head buffers and, with `layers` (training), the activation buffers for T tours
// of length n (padding rows cleared for this n). Growing waits for enqueued work.
split_status ensure_act(split_nn *nn, int32_t T, int32_t n, bool layers, hipStream_t st)
{
    const int64_t rows = layers ? (int64_t)T * (n + 4) : 0;
    if (rows > nn->cap_rows) {
        NN_TRY(nn, hipDeviceSynchronize());
        const int64_t cap = rows + rows / 4;
        nn->cap_rows = 0;
        bool ok = realloc_dev(&nn->X, sizeof(uint16_t) * cap * kNnCi0);
        for (int l = 0; l < 4; ++l) ok = ok && realloc_dev(&nn->H[l], sizeof(uint16_t) * cap * kNnWidth);
        for (int k = 0; k < 2; ++k) ok = ok && realloc_dev(&nn->dP[k], sizeof(uint16_t) * cap * kNnWidth);
        if (!ok) return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "surrogate: activation buffers failed");
        nn->cap_rows = cap;
        nn->zero_n = -1;
    }
    if (layers && nn->zero_n != n) {
        // padding rows are never written by the kernels: clear whole buffers for this layout
        NN_TRY(nn, hipMemsetAsync(nn->X, 0, sizeof(uint16_t) * nn->cap_rows * kNnCi0, st));
        for (int l = 0; l < 4; ++l)
            NN_TRY(nn, hipMemsetAsync(nn->H[l], 0, sizeof(uint16_t) * nn->cap_rows * kNnWidth, st));
        for (int k = 0; k < 2; ++k)
            NN_TRY(nn, hipMemsetAsync(nn->dP[k], 0, sizeof(uint16_t) * nn->cap_rows * kNnWidth, st));
        nn->zero_n = n;
    }
    if (T > nn->cap_T) {
        NN_TRY(nn, hipDeviceSynchronize());
        const int32_t cap = T < 64 ? 64 : T;
        nn->cap_T = 0;
        bool ok = true;
        for (float **p : {&nn->z, &nn->a, &nn->da, &nn->dz})
            ok = ok && realloc_dev(p, sizeof(float) * (size_t)cap * kNnWidth);
        for (float **p : {&nn->y, &nn->dy, &nn->lterms})
            ok = ok && realloc_dev(p, sizeof(float) * (size_t)cap);
        if (!ok) return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "surrogate: head buffers failed");
        nn->cap_T = cap;
    }
    return SPLIT_OK;
}

split_status check_call(split_nn *nn, const char *who, const void *tours, int32_t T, int32_t n,
                        NnInstance *in)
{
    if (!tours) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "%s: NULL tours", who);
    if (!nn->have_scen)
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "%s: no scenario set (split_nn_set_scenarios)",
                        who);
    int64_t max_arc = 0;
    if (!instance_of(nn, in, &max_arc))
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "%s: no instance set", who);
    if (in->N != nn->musd_N)
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "%s: the instance changed since "
                        "split_nn_set_scenarios", who);
    if (T < 1 || n < 1 || n > in->N)
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "%s: need T >= 1 and 1 <= n <= N", who);
    return SPLIT_OK;
}

// Features, the four conv layers and the head for T tours. With pred (prediction) the layers
// run fused per tile in LDS; without (training) every layer's output is kept for backward.
constexpr size_t kMaxTimingPairs = 4096;

split_status collect_timing(split_nn *nn)
{
    for (size_t k = 0; k < nn->tpairs_used; ++k) {
        NN_TRY(nn, hipEventSynchronize(nn->tpairs[k].second));
        float ms = 0.f;
        NN_TRY(nn, hipEventElapsedTime(&ms, nn->tpairs[k].first, nn->tpairs[k].second));
        nn->ms_acc += ms;
        nn->launches += 1;
    }
    nn->tpairs_used = 0;
    return SPLIT_OK;
}

// Records the start event of a timed launch on st and hands back its stop event (nullptr when
// timing is off).
split_status timing_begin(split_nn *nn, hipStream_t st, hipEvent_t *stop)
{
    *stop = nullptr;
    if (!nn->timing) return SPLIT_OK;
    if (nn->tpairs_used == kMaxTimingPairs) {
        split_status s = collect_timing(nn);
        if (s != SPLIT_OK) return s;
    }
    if (nn->tpairs_used == nn->tpairs.size()) {
        hipEvent_t a, b;
        NN_TRY(nn, hipEventCreate(&a));
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return ctx_fail(nn->ctx, SPLIT_E_HIP, "surrogate: timing event failed");
        }
        nn->tpairs.emplace_back(a, b);
    }
    auto &pr = nn->tpairs[nn->tpairs_used++];
    NN_TRY(nn, hipEventRecord(pr.first, st));
    *stop = pr.second;
    return SPLIT_OK;
}

split_status forward(split_nn *nn, const NnInstance &in, const int32_t *tours, int32_t T,
                     int32_t n, float *pred, hipStream_t st)
{
    split_status s = ensure_act(nn, T, n, pred == nullptr, st);
    if (s != SPLIT_OK) return s;
    if (pred) {
        const int64_t need = (int64_t)T * nn_fused_tiles(n) * kNnWidth;
        if (need > nn->cap_zpart) {
            NN_TRY(nn, hipDeviceSynchronize());
            nn->cap_zpart = 0;
            if (!realloc_dev(&nn->zpart, sizeof(float) * (size_t)need))
                return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "surrogate: pooling buffer failed");
            nn->cap_zpart = need;
        }
        const int64_t pos = (int64_t)T * n;
        if (pos > nn->cap_xp) {
            NN_TRY(nn, hipDeviceSynchronize());
            const int64_t cap = pos + pos / 4;
            nn->cap_xp = 0;
            if (!realloc_dev(&nn->Xp, sizeof(uint16_t) * kNnFeatures * (size_t)cap))
                return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "surrogate: packed feature buffer failed");
            nn->cap_xp = cap;
        }
        NN_TRY(nn, nn_launch_features(in, tours, T, n, nn->musd, nn->Q, nn->L, nn->Xp, true,
                                      nn->err, st));
        hipEvent_t stop = nullptr;
        s = timing_begin(nn, st, &stop);
        if (s != SPLIT_OK) return s;
        NN_TRY(nn, nn_launch_fwd_fused(nn->Xp, nn->w, nn->P, T, n, nn->zpart, st));
        if (stop) NN_TRY(nn, hipEventRecord(stop, st));
        NN_TRY(nn, nn_launch_head_pool(nn->zpart, T, n, nn->P, nn->z, nn->a, nn->y, pred,
                                       nn->shift, nn->scale, st));
        return SPLIT_OK;
    }
    NN_TRY(nn, nn_launch_features(in, tours, T, n, nn->musd, nn->Q, nn->L, nn->X, false, nn->err,
                                  st));
    NN_TRY(nn, nn_launch_conv(kNnCi0, 0, nn->X, nn->w.f[0], nn->P + nn_off_b(0), nullptr, nn->H[0],
                              T, n, st));
    for (int l = 1; l < 4; ++l)
        NN_TRY(nn, nn_launch_conv(kNnWidth, 0, nn->H[l - 1], nn->w.f[l], nn->P + nn_off_b(l),
                                  nullptr, nn->H[l], T, n, st));
    NN_TRY(nn, nn_launch_head_fwd(nn->H[3], T, n, nn->P, nn->z, nn->a, nn->y, pred, nn->shift,
                                  nn->scale, st));
    return SPLIT_OK;
}

// Loss terms and the full gradient into nn->G for the batch whose forward pass just ran.
split_status backward(split_nn *nn, const float *labels, int32_t T, int32_t n, hipStream_t st)
{
    const int64_t chunks = nn_wgrad_chunks(T, n, kWgradChunk);
    if (chunks > nn->cap_chunks) {
        NN_TRY(nn, hipDeviceSynchronize());
        nn->cap_chunks = 0;
        if (!realloc_dev(&nn->partW, sizeof(float) * (size_t)chunks * kNnSizeWl) ||
            !realloc_dev(&nn->partB, sizeof(float) * (size_t)chunks * kNnWidth))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "surrogate: gradient partials failed");
        nn->cap_chunks = chunks;
    }
    NN_TRY(nn, nn_launch_head_bwd(labels, T, n, nn->P, nn->z, nn->a, nn->y, nn->shift, nn->scale,
                                  nn->da, nn->dz, nn->dy, nn->lterms, nn->H[3], nn->dP[0], nn->G,
                                  st));
    // layer l (0-based) reads input in[l] and the pre-activation gradient cur; for l > 0 the
    // input gradient goes into the other dP buffer
    const uint16_t *in_of[4] = {nn->X, nn->H[0], nn->H[1], nn->H[2]};
    int cur = 0;
    for (int l = 3; l >= 0; --l) {
        NN_TRY(nn, nn_launch_wgrad(l == 0 ? kNnCi0 : kNnWidth, in_of[l], nn->dP[cur], T, n,
                                   kWgradChunk, (int32_t)chunks, nn->partW, nn->partB, nn->G,
                                   nn_off_w(l), nn_off_b(l), st));
        if (l > 0) {
            NN_TRY(nn, nn_launch_conv(kNnWidth, 1, nn->dP[cur], nn->w.b[l], nullptr, in_of[l],
                                      nn->dP[1 - cur], T, n, st));
            cur = 1 - cur;
        }
    }
    return SPLIT_OK;
}

split_status adam_step(split_nn *nn, float lr, hipStream_t st)
{
    nn->step += 1;
    const float bc1 = (float)(1.0 - pow(0.9, (double)nn->step));
    const float bc2 = (float)(1.0 - pow(0.999, (double)nn->step));
    NN_TRY(nn, nn_launch_adam(nn->P, nn->m, nn->v, nn->G, lr, bc1, bc2, st));
    NN_TRY(nn, nn_launch_pack(nn->P, nn->w, st));
    return SPLIT_OK;
}

// Waits for the stream and fails with SPLIT_E_TOUR if a feature kernel met a bad id.
split_status check_ids(split_nn *nn, const char *who, hipStream_t st)
{
    NN_TRY(nn, hipMemcpyAsync(nn->h_err, nn->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    NN_TRY(nn, hipStreamSynchronize(st));
    if (*nn->h_err)
        return ctx_fail(nn->ctx, SPLIT_E_TOUR, "%s: a tour id is outside 1..N", who);
    return SPLIT_OK;
}

split_status topk_run(split_ctx *ctx, TopkScratch &k, const float *scores, int64_t C, int64_t K,
                      int32_t *idx, hipStream_t st)
{
    const int64_t nb = (C + 255) / 256;
    if (!k.sel || nb > k.cap_blocks) {
        if (hipDeviceSynchronize() != hipSuccess)
            return ctx_fail(ctx, SPLIT_E_HIP, "top-k: hipDeviceSynchronize failed");
        free_topk(k);
        if (hipMalloc(&k.sel, sizeof(NnSelect)) != hipSuccess ||
            hipMalloc(&k.hist, sizeof(unsigned long long) * 256) != hipSuccess ||
            hipMalloc(&k.cnt, sizeof(unsigned int) * 2 * (size_t)nb) != hipSuccess ||
            hipMalloc(&k.base, sizeof(unsigned long long) * 2 * (size_t)nb) != hipSuccess)
            return ctx_fail(ctx, SPLIT_E_NOMEM, "top-k: scratch allocation failed");
        k.cap_blocks = nb;
    }
    NnSelect init = {0u, 0u, (unsigned long long)K};
    if (hipMemcpyAsync(k.sel, &init, sizeof init, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(k.hist, 0, sizeof(unsigned long long) * 256, st) != hipSuccess)
        return ctx_fail(ctx, SPLIT_E_HIP, "top-k: setup copies failed");
    const hipError_t e = nn_launch_topk(scores, C, K, k.sel, k.hist, k.cnt, k.base, idx, st);
    if (e != hipSuccess) return ctx_fail(ctx, SPLIT_E_HIP, "top-k: %s", hipGetErrorString(e));
    // the init struct lives on this stack frame: finish before returning
    if (hipStreamSynchronize(st) != hipSuccess)
        return ctx_fail(ctx, SPLIT_E_HIP, "top-k: hipStreamSynchronize failed");
    return SPLIT_OK;
}

void free_nn(split_nn *nn)
{
    for (float *p : {nn->P, nn->m, nn->v, nn->G, nn->z, nn->a, nn->y, nn->da, nn->dz, nn->dy,
                     nn->lterms, nn->lout, nn->partW, nn->partB, nn->blabels, nn->losshist,
                     nn->pred, nn->zpart})
        if (p) (void)hipFree(p);
    for (int l = 0; l < 4; ++l) {
        if (nn->w.f[l]) (void)hipFree(nn->w.f[l]);
        if (nn->w.b[l]) (void)hipFree(nn->w.b[l]);
        if (nn->w.g[l]) (void)hipFree(nn->w.g[l]);
        if (nn->H[l]) (void)hipFree(nn->H[l]);
    }
    for (uint16_t *p : {nn->X, nn->Xp, nn->dP[0], nn->dP[1]})
        if (p) (void)hipFree(p);
    for (int32_t *p : {nn->err, nn->btours, nn->perm, nn->sidx, nn->stours, nn->ecost})
        if (p) (void)hipFree(p);
    if (nn->musd) (void)hipFree(nn->musd);
    if (nn->h_err) (void)hipHostFree(nn->h_err);
    free_topk(nn->tk);
    for (auto &pr : nn->tpairs) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    nn->tpairs.clear();
}

// He-uniform weights from the seed, zero biases.
void init_params(std::vector<float> &p, uint64_t seed)
{
    p.assign(kNnParams, 0.f);
    uint64_t s = seed;
    auto fill = [&](int off, int count, double fan_in, int ci_stride, int ci_live) {
        const double a = sqrt(6.0 / fan_in);
        for (int e = 0; e < count; ++e) {
            const double u = uniform01(s);
            // W1: input channels past the 8 features stay zero
            const bool live = ci_stride == 0 || (e / ci_stride) % kNnCi0 < ci_live;
            p[off + e] = live ? (float)((2.0 * u - 1.0) * a) : 0.f;
        }
    };
    fill(nn_off_w(0), kNnSizeW1, kNnTaps * 8.0, kNnWidth, 8);
    for (int l = 1; l < 4; ++l) fill(nn_off_w(l), kNnSizeWl, kNnTaps * (double)kNnWidth, 0, 0);
    fill(kNnOffWa, kNnWidth * kNnWidth, kNnWidth, 0, 0);
    fill(kNnOffWb, kNnWidth, kNnWidth, 0, 0);
}

split_status upload_params(split_nn *nn, const float *host)
{
    NN_TRY(nn, hipMemcpy(nn->P, host, sizeof(float) * kNnParams, hipMemcpyHostToDevice));
    NN_TRY(nn, hipMemset(nn->m, 0, sizeof(float) * kNnParams));
    NN_TRY(nn, hipMemset(nn->v, 0, sizeof(float) * kNnParams));
    NN_TRY(nn, nn_launch_pack(nn->P, nn->w, nullptr));
    NN_TRY(nn, hipDeviceSynchronize());
    nn->step = 0;
    return SPLIT_OK;
}

struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t nparams;
    int64_t step;
    double shift, scale, L;
};

}  // namespace

extern "C" {

split_status split_nn_create(split_ctx *ctx, uint64_t seed, double length_scale, split_nn **out)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!out) return ctx_fail(ctx, SPLIT_E_INVAL, "split_nn_create: NULL out");
    *out = nullptr;
    if (!(length_scale > 0.0))
        return ctx_fail(ctx, SPLIT_E_INVAL, "split_nn_create: length_scale must be > 0");
    split_nn *nn = new (std::nothrow) split_nn();
    if (!nn) return ctx_fail(ctx, SPLIT_E_NOMEM, "split_nn_create: out of host memory");
    nn->ctx = ctx;
    nn->device = ctx_device(ctx);
    nn->L = length_scale;
    Guard g(nn->device);
    bool ok = g.ok;
    for (float **p : {&nn->P, &nn->m, &nn->v, &nn->G})
        ok = ok && hipMalloc(p, sizeof(float) * kNnParams) == hipSuccess;
    ok = ok && hipMalloc(&nn->w.f[0], sizeof(uint16_t) * kNnSizeW1) == hipSuccess &&
         hipMalloc(&nn->w.g[0], sizeof(uint16_t) * kNnSizeW1) == hipSuccess &&
         // the fused kernel's packed layer-1 weights: padding entries are never written
         hipMemset(nn->w.g[0], 0, sizeof(uint16_t) * kNnSizeW1) == hipSuccess;
    for (int l = 1; l < 4; ++l)
        ok = ok && hipMalloc(&nn->w.f[l], sizeof(uint16_t) * kNnSizeWl) == hipSuccess &&
             hipMalloc(&nn->w.b[l], sizeof(uint16_t) * kNnSizeWl) == hipSuccess &&
             hipMalloc(&nn->w.g[l], sizeof(uint16_t) * kNnSizeWl) == hipSuccess;
    ok = ok && hipMalloc(&nn->err, sizeof(int32_t)) == hipSuccess &&
         hipMalloc(&nn->lout, sizeof(float)) == hipSuccess &&
         hipHostMalloc((void **)&nn->h_err, sizeof(int32_t), 0) == hipSuccess;
    if (!ok) {
        free_nn(nn);
        delete nn;
        return ctx_fail(ctx, SPLIT_E_NOMEM, "split_nn_create: device allocation failed");
    }
    std::vector<float> p;
    init_params(p, seed);
    split_status st = upload_params(nn, p.data());
    if (st != SPLIT_OK) {
        free_nn(nn);
        delete nn;
        return st;
    }
    *out = nn;
    return SPLIT_OK;
}

void split_nn_destroy(split_nn *nn)
{
    if (!nn) return;
    {
        Guard g(nn->device);
        (void)hipDeviceSynchronize();
        free_nn(nn);
    }
    delete nn;
}

split_status split_nn_params_get(split_nn *nn, float *params)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!params) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_params_get: NULL params");
    Guard g(nn->device);
    NN_TRY(nn, hipDeviceSynchronize());
    NN_TRY(nn, hipMemcpy(params, nn->P, sizeof(float) * kNnParams, hipMemcpyDeviceToHost));
    return SPLIT_OK;
}

split_status split_nn_params_set(split_nn *nn, const float *params)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!params) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_params_set: NULL params");
    for (int64_t e = 0; e < kNnParams; ++e)
        if (!isfinite(params[e]))
            return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_params_set: parameter %lld is not "
                            "finite", (long long)e);
    Guard g(nn->device);
    NN_TRY(nn, hipDeviceSynchronize());
    return upload_params(nn, params);
}

split_status split_nn_set_norm(split_nn *nn, double shift, double scale)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!(scale > 0.0) || !isfinite(shift) || !isfinite(scale))
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_set_norm: need finite shift, scale > 0");
    nn->shift = shift;
    nn->scale = scale;
    return SPLIT_OK;
}

split_status split_nn_set_scenarios(split_nn *nn, const int16_t *demand, int64_t S, int64_t ld,
                                    int32_t Q)
{
    if (!nn) return SPLIT_E_INVAL;
    NnInstance in;
    int64_t max_arc = 0;
    if (!instance_of(nn, &in, &max_arc))
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_set_scenarios: no instance set");
    if (!demand || S < 1 || ld < S || Q < 1)
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_set_scenarios: need demand, 1 <= S <= "
                        "ld, Q >= 1");
    Guard g(nn->device);
    NN_TRY(nn, hipDeviceSynchronize());
    if (in.N > nn->musd_N || !nn->musd) {
        if (!realloc_dev(&nn->musd, sizeof(double) * 2 * (size_t)in.N))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_set_scenarios: allocation failed");
    }
    NN_TRY(nn, nn_launch_dstats(demand, ld, S, in.N, nn->musd, nullptr));
    NN_TRY(nn, hipDeviceSynchronize());
    nn->musd_N = in.N;
    nn->Q = Q;
    nn->have_scen = true;
    return SPLIT_OK;
}

split_status split_nn_predict(split_nn *nn, const int32_t *tours, int32_t T, int32_t n,
                              float *pred, void *hip_stream)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!pred) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_predict: NULL pred");
    NnInstance in;
    split_status s = check_call(nn, "split_nn_predict", tours, T, n, &in);
    if (s != SPLIT_OK) return s;
    Guard g(nn->device);
    hipStream_t st = (hipStream_t)hip_stream;
    NN_TRY(nn, hipMemsetAsync(nn->err, 0, sizeof(int32_t), st));
    for (int32_t t0 = 0; t0 < T; t0 += kPredChunk) {
        const int32_t Tc = T - t0 < kPredChunk ? T - t0 : kPredChunk;
        s = forward(nn, in, tours + (int64_t)t0 * n, Tc, n, pred + t0, st);
        if (s != SPLIT_OK) return s;
    }
    return check_ids(nn, "split_nn_predict", st);
}

split_status split_nn_gradient(split_nn *nn, const int32_t *tours, const float *labels,
                               int32_t T, int32_t n, float *grad, double *loss, void *hip_stream)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!labels) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_gradient: NULL labels");
    NnInstance in;
    split_status s = check_call(nn, "split_nn_gradient", tours, T, n, &in);
    if (s != SPLIT_OK) return s;
    Guard g(nn->device);
    hipStream_t st = (hipStream_t)hip_stream;
    NN_TRY(nn, hipMemsetAsync(nn->err, 0, sizeof(int32_t), st));
    s = forward(nn, in, tours, T, n, nullptr, st);
    if (s == SPLIT_OK) s = backward(nn, labels, T, n, st);
    if (s != SPLIT_OK) return s;
    NN_TRY(nn, nn_launch_loss(nn->lterms, T, nn->lout, st));
    s = check_ids(nn, "split_nn_gradient", st);
    if (s != SPLIT_OK) return s;
    if (grad) NN_TRY(nn, hipMemcpy(grad, nn->G, sizeof(float) * kNnParams, hipMemcpyDeviceToHost));
    if (loss) {
        float l = 0.f;
        NN_TRY(nn, hipMemcpy(&l, nn->lout, sizeof(float), hipMemcpyDeviceToHost));
        *loss = l;
    }
    return SPLIT_OK;
}

split_status split_nn_train_step(split_nn *nn, const int32_t *tours, const float *labels,
                                 int32_t T, int32_t n, float lr, double *loss,
                                 void *hip_stream)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!labels || !(lr > 0.f))
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_train_step: need labels and lr > 0");
    NnInstance in;
    split_status s = check_call(nn, "split_nn_train_step", tours, T, n, &in);
    if (s != SPLIT_OK) return s;
    Guard g(nn->device);
    hipStream_t st = (hipStream_t)hip_stream;
    NN_TRY(nn, hipMemsetAsync(nn->err, 0, sizeof(int32_t), st));
    s = forward(nn, in, tours, T, n, nullptr, st);
    if (s == SPLIT_OK) s = backward(nn, labels, T, n, st);
    if (s != SPLIT_OK) return s;
    NN_TRY(nn, nn_launch_loss(nn->lterms, T, nn->lout, st));
    // ids are checked before the update touches the parameters
    s = check_ids(nn, "split_nn_train_step", st);
    if (s != SPLIT_OK) return s;
    s = adam_step(nn, lr, st);
    if (s != SPLIT_OK) return s;
    if (loss) {
        float l = 0.f;
        NN_TRY(nn, hipMemcpy(&l, nn->lout, sizeof(float), hipMemcpyDeviceToHost));
        *loss = l;
    }
    return SPLIT_OK;
}

split_status split_nn_train(split_nn *nn, const int32_t *tours, const float *labels,
                            int64_t count, int32_t n, int32_t batch, int64_t steps, float lr,
                            uint64_t seed, double *mean_loss, void *hip_stream)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!labels || batch < 1 || count < batch || count > INT32_MAX || steps < 0 || !(lr > 0.f))
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_train: need labels, 1 <= batch <= count "
                        "< 2^31, steps >= 0, lr > 0");
    NnInstance in;
    split_status s = check_call(nn, "split_nn_train", tours, batch, n, &in);
    if (s != SPLIT_OK) return s;
    Guard g(nn->device);
    hipStream_t st = (hipStream_t)hip_stream;
    // every id of the training set, once, before any update
    NN_TRY(nn, hipMemsetAsync(nn->err, 0, sizeof(int32_t), st));
    NN_TRY(nn, nn_launch_check_ids(tours, count * n, in.N, nn->err, st));
    s = check_ids(nn, "split_nn_train", st);
    if (s != SPLIT_OK) return s;
    NN_TRY(nn, hipDeviceSynchronize());
    if ((int64_t)batch * n > nn->cap_btours) {
        if (!realloc_dev(&nn->btours, sizeof(int32_t) * (size_t)batch * n))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_train: batch buffer failed");
        nn->cap_btours = (int64_t)batch * n;
    }
    if (batch > nn->cap_blab) {
        if (!realloc_dev(&nn->blabels, sizeof(float) * (size_t)batch))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_train: label buffer failed");
        nn->cap_blab = batch;
    }
    if (count > nn->cap_perm) {
        if (!realloc_dev(&nn->perm, sizeof(int32_t) * (size_t)count))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_train: permutation buffer failed");
        nn->cap_perm = count;
    }
    if (steps > nn->cap_losshist) {
        if (!realloc_dev(&nn->losshist, sizeof(float) * (size_t)steps))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_train: loss buffer failed");
        nn->cap_losshist = steps;
    }
    const int64_t bpe = count / batch;
    std::vector<int32_t> perm((size_t)count);
    int64_t perm_epoch = -1;
    for (int64_t k = 0; k < steps; ++k) {
        const int64_t b = nn->step;
        const int64_t epoch = b / bpe, pos = b % bpe;
        if (epoch != perm_epoch) {
            // Fisher-Yates with a stream keyed by (seed, epoch)
            uint64_t rs = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(epoch + 1));
            for (int64_t i = 0; i < count; ++i) perm[i] = (int32_t)i;
            for (int64_t i = count - 1; i > 0; --i) {
                const int64_t j = (int64_t)(splitmix64(rs) % (uint64_t)(i + 1));
                const int32_t tmp = perm[i];
                perm[i] = perm[j];
                perm[j] = tmp;
            }
            NN_TRY(nn, hipStreamSynchronize(st));  // the previous epoch's gathers are done
            NN_TRY(nn, hipMemcpy(nn->perm, perm.data(), sizeof(int32_t) * (size_t)count,
                                 hipMemcpyHostToDevice));
            perm_epoch = epoch;
        }
        NN_TRY(nn, nn_launch_gather(tours, labels, nn->perm + pos * batch, batch, n, nn->btours,
                                    nn->blabels, st));
        s = forward(nn, in, nn->btours, batch, n, nullptr, st);
        if (s == SPLIT_OK) s = backward(nn, nn->blabels, batch, n, st);
        if (s != SPLIT_OK) return s;
        NN_TRY(nn, nn_launch_loss(nn->lterms, batch, nn->losshist + k, st));
        s = adam_step(nn, lr, st);
        if (s != SPLIT_OK) return s;
    }
    NN_TRY(nn, hipStreamSynchronize(st));
    if (mean_loss) {
        std::vector<float> lh((size_t)steps);
        if (steps > 0)
            NN_TRY(nn, hipMemcpy(lh.data(), nn->losshist, sizeof(float) * (size_t)steps,
                                 hipMemcpyDeviceToHost));
        double sum = 0.0;
        for (float x : lh) sum += x;
        *mean_loss = steps > 0 ? sum / (double)steps : 0.0;
    }
    return SPLIT_OK;
}

split_status split_nn_step(split_nn *nn, int64_t *step)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!step) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_step: NULL step");
    *step = nn->step;
    return SPLIT_OK;
}

split_status split_nn_save(split_nn *nn, const char *path)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!path) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_save: NULL path");
    Guard g(nn->device);
    NN_TRY(nn, hipDeviceSynchronize());
    std::vector<float> buf(3 * (size_t)kNnParams);
    NN_TRY(nn, hipMemcpy(buf.data(), nn->P, sizeof(float) * kNnParams, hipMemcpyDeviceToHost));
    NN_TRY(nn, hipMemcpy(buf.data() + kNnParams, nn->m, sizeof(float) * kNnParams,
                         hipMemcpyDeviceToHost));
    NN_TRY(nn, hipMemcpy(buf.data() + 2 * (size_t)kNnParams, nn->v, sizeof(float) * kNnParams,
                         hipMemcpyDeviceToHost));
    CkptHeader h;
    memcpy(h.magic, kMagic, 8);
    h.version = 1;
    h.nparams = kNnParams;
    h.step = nn->step;
    h.shift = nn->shift;
    h.scale = nn->scale;
    h.L = nn->L;
    FILE *f = fopen(path, "wb");
    if (!f) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_save: cannot open %s", path);
    const bool ok = fwrite(&h, sizeof h, 1, f) == 1 &&
                    fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    if (fclose(f) != 0 || !ok)
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_save: write to %s failed", path);
    return SPLIT_OK;
}

split_status split_nn_load(split_nn *nn, const char *path)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!path) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_load: NULL path");
    FILE *f = fopen(path, "rb");
    if (!f) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_load: cannot open %s", path);
    CkptHeader h;
    std::vector<float> buf(3 * (size_t)kNnParams);
    bool ok = fread(&h, sizeof h, 1, f) == 1 && memcmp(h.magic, kMagic, 8) == 0 &&
              h.version == 1 && h.nparams == (uint32_t)kNnParams && h.step >= 0 &&
              h.scale > 0.0 && h.L > 0.0 &&
              fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_load: %s is not a surrogate "
                             "checkpoint of this layout", path);
    Guard g(nn->device);
    NN_TRY(nn, hipDeviceSynchronize());
    NN_TRY(nn, hipMemcpy(nn->P, buf.data(), sizeof(float) * kNnParams, hipMemcpyHostToDevice));
    NN_TRY(nn, hipMemcpy(nn->m, buf.data() + kNnParams, sizeof(float) * kNnParams,
                         hipMemcpyHostToDevice));
    NN_TRY(nn, hipMemcpy(nn->v, buf.data() + 2 * (size_t)kNnParams, sizeof(float) * kNnParams,
                         hipMemcpyHostToDevice));
    NN_TRY(nn, nn_launch_pack(nn->P, nn->w, nullptr));
    NN_TRY(nn, hipDeviceSynchronize());
    nn->step = h.step;
    nn->shift = h.shift;
    nn->scale = h.scale;
    nn->L = h.L;
    return SPLIT_OK;
}

split_status split_topk_smallest(split_ctx *ctx, const float *scores, int64_t C, int64_t K,
                                 int32_t *idx, void *hip_stream)
{
    if (!ctx) return SPLIT_E_INVAL;
    if (!scores || !idx || K < 1 || K > C || C >= ((int64_t)1 << 31))
        return ctx_fail(ctx, SPLIT_E_INVAL, "split_topk_smallest: need scores, idx and "
                        "1 <= K <= C < 2^31");
    Guard g(ctx_device(ctx));
    TopkScratch k;
    const split_status s = topk_run(ctx, k, scores, C, K, idx, (hipStream_t)hip_stream);
    free_topk(k);
    return s;
}

split_status split_nn_shortlist(split_nn *nn, const int32_t *tours, int32_t T, int32_t n,
                                int32_t K, int32_t *idx, float *pred, void *hip_stream)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!idx || K < 1 || K > T)
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_shortlist: need idx and 1 <= K <= T");
    NnInstance in;
    split_status s = check_call(nn, "split_nn_shortlist", tours, T, n, &in);
    if (s != SPLIT_OK) return s;
    Guard g(nn->device);
    hipStream_t st = (hipStream_t)hip_stream;
    float *pr = pred;
    if (!pr) {
        if (T > nn->cap_pred) {
            NN_TRY(nn, hipDeviceSynchronize());
            if (!realloc_dev(&nn->pred, sizeof(float) * (size_t)T))
                return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_shortlist: prediction buffer");
            nn->cap_pred = T;
        }
        pr = nn->pred;
    }
    NN_TRY(nn, hipMemsetAsync(nn->err, 0, sizeof(int32_t), st));
    for (int32_t t0 = 0; t0 < T; t0 += kPredChunk) {
        const int32_t Tc = T - t0 < kPredChunk ? T - t0 : kPredChunk;
        s = forward(nn, in, tours + (int64_t)t0 * n, Tc, n, pr + t0, st);
        if (s != SPLIT_OK) return s;
    }
    s = check_ids(nn, "split_nn_shortlist", st);
    if (s != SPLIT_OK) return s;
    return topk_run(nn->ctx, nn->tk, pr, T, K, idx, st);
}

split_status split_nn_screen(split_nn *nn, const int32_t *cands, int64_t C, int32_t n, int64_t K,
                             const int16_t *demand, int64_t S, int64_t ld, int32_t Q,
                             float *pred, int32_t *short_idx, double *short_mean,
                             int64_t *best_idx, double *best_mean, void *hip_stream)
{
    if (!nn) return SPLIT_E_INVAL;
    if (!best_idx || !best_mean || K < 1 || K > C || C >= ((int64_t)1 << 31))
        return ctx_fail(nn->ctx, SPLIT_E_INVAL, "split_nn_screen: need best_idx, best_mean and "
                        "1 <= K <= C < 2^31");
    NnInstance in;
    split_status s = check_call(nn, "split_nn_screen", cands, 1, n, &in);
    if (s != SPLIT_OK) return s;
    Guard g(nn->device);
    hipStream_t st = (hipStream_t)hip_stream;
    float *pr = pred;
    if (!pr) {
        if (C > nn->cap_pred) {
            NN_TRY(nn, hipDeviceSynchronize());
            if (!realloc_dev(&nn->pred, sizeof(float) * (size_t)C))
                return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_screen: prediction buffer");
            nn->cap_pred = C;
        }
        pr = nn->pred;
    }
    NN_TRY(nn, hipMemsetAsync(nn->err, 0, sizeof(int32_t), st));
    for (int64_t t0 = 0; t0 < C; t0 += kPredChunk) {
        const int32_t Tc = (int32_t)(C - t0 < kPredChunk ? C - t0 : kPredChunk);
        s = forward(nn, in, cands + t0 * n, Tc, n, pr + t0, st);
        if (s != SPLIT_OK) return s;
    }
    s = check_ids(nn, "split_nn_screen", st);
    if (s != SPLIT_OK) return s;
    if (K > nn->cap_sidx || K * n > nn->cap_stours) {
        NN_TRY(nn, hipDeviceSynchronize());
        if (!realloc_dev(&nn->sidx, sizeof(int32_t) * (size_t)K) ||
            !realloc_dev(&nn->stours, sizeof(int32_t) * (size_t)K * n))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_screen: shortlist buffers");
        nn->cap_sidx = K;
        nn->cap_stours = K * n;
    }
    s = topk_run(nn->ctx, nn->tk, pr, C, K, nn->sidx, st);
    if (s != SPLIT_OK) return s;
    NN_TRY(nn, nn_launch_gather(cands, nullptr, nn->sidx, (int32_t)K, n, nn->stours, nullptr, st));
    std::vector<int32_t> hidx((size_t)K), htours((size_t)K * n);
    NN_TRY(nn, hipMemcpyAsync(hidx.data(), nn->sidx, sizeof(int32_t) * (size_t)K,
                              hipMemcpyDeviceToHost, st));
    NN_TRY(nn, hipMemcpyAsync(htours.data(), nn->stours, sizeof(int32_t) * (size_t)K * n,
                              hipMemcpyDeviceToHost, st));
    NN_TRY(nn, hipStreamSynchronize(st));
    // exact means of the shortlist, kExactChunk tours per batch evaluation
    const int64_t need = (int64_t)kExactChunk * S;
    if (need > nn->cap_ecost) {
        NN_TRY(nn, hipDeviceSynchronize());
        if (!realloc_dev(&nn->ecost, sizeof(int32_t) * (size_t)need))
            return ctx_fail(nn->ctx, SPLIT_E_NOMEM, "split_nn_screen: cost buffer");
        nn->cap_ecost = need;
    }
    std::vector<split_stats> stats(kExactChunk);
    std::vector<int64_t> ptr(kExactChunk + 1);
    int64_t bi = -1;
    double bm = 0.0;
    for (int64_t k0 = 0; k0 < K; k0 += kExactChunk) {
        const int32_t Tc = (int32_t)(K - k0 < kExactChunk ? K - k0 : kExactChunk);
        for (int32_t t = 0; t <= Tc; ++t) ptr[t] = (int64_t)t * n;
        s = split_eval_batch(nn->ctx, htours.data() + k0 * n, ptr.data(), Tc, demand, S, ld, Q,
                             nn->ecost, S, stats.data(), nullptr, hip_stream);
        if (s != SPLIT_OK) return s;
        for (int32_t t = 0; t < Tc; ++t) {
            if (short_mean) short_mean[k0 + t] = stats[t].mean;
            if (bi < 0 || stats[t].mean < bm) {
                bi = hidx[k0 + t];
                bm = stats[t].mean;
            }
        }
    }
    if (short_idx) memcpy(short_idx, hidx.data(), sizeof(int32_t) * (size_t)K);
    *best_idx = bi;
    *best_mean = bm;
    return SPLIT_OK;
}

split_status split_nn_timing_enable(split_nn *nn, int enable)
{
    if (!nn) return SPLIT_E_INVAL;
    nn->timing = enable != 0;
    return SPLIT_OK;
}

split_status split_nn_timing_get(split_nn *nn, double *ms_total, int64_t *launches)
{
    if (!nn) return SPLIT_E_INVAL;
    Guard g(nn->device);
    split_status s = collect_timing(nn);
    if (s != SPLIT_OK) return s;
    if (ms_total) *ms_total = nn->ms_acc;
    if (launches) *launches = nn->launches;
    return SPLIT_OK;
}

split_status split_nn_timing_reset(split_nn *nn)
{
    if (!nn) return SPLIT_E_INVAL;
    Guard g(nn->device);
    split_status s = collect_timing(nn);
    nn->ms_acc = 0.0;
    nn->launches = 0;
    return s;
}

}  // extern "C"
