// HIP kernels for the scenario-batched Split (arXiv 2511.18022, Section 3) on gfx950.
//
// Notation (Section 3): positions 1..n of the giant tour s_1..s_n, DP states f(0..n),
// capacity window of state i = predecessors p in [mask(i), i-1] (Eq. (2)), Eq. (3) minimum
// over that window. The route cost of segment p+1..i splits into a term of p and a term of i,
// so with
//     g_p = f_p + c(0, s_{p+1}) - D[p+1]       (D[k] = sum of tour arcs up to position k)
// Eq. (3) becomes a sliding-window minimum:  g_i = w_i + min_{p in window(i)} g_p,
// where w_i depends on the tour only (built by split_prep_kernel) and f_n = g_n.
// All DP arithmetic is int32 and exact.
//
// Kernels:
//  split_prep_kernel      per-tour w_i and demand row offsets; zeroes the result block.
//  split_lane_kernel      one scenario per lane (scenario-level parallelism of Section 3);
//                         the window minimum is answered in O(1) per state from block
//                         suffix minima held in LDS; windows longer than its LDS history are
//                         queued for the general kernel.
//  split_wave_kernel      one scenario per wavefront; lanes cover the window's predecessors
//                         (transition-level parallelism of Section 3) and the minimum is a
//                         DPP reduction. Exact for any window length; used for small S and
//                         for the scenarios the lane kernel queues.
//  split_moments_*        exact 128-bit sum and sum of squares of the costs.
#include "split_internal.h"

namespace splitgpu {

// ------------------------------------------------------------------------- distances

// Nearest integer to the Euclidean distance between integer points (|coord| <= 2^20, so
// m < 2^43 and the double square root is within one unit of floor(sqrt(m))).
__device__ __forceinline__ int32_t dist_coords(const int32_t *xy, int u, int v)
{
    const long long dx = (long long)xy[2 * u] - xy[2 * v];
    const long long dy = (long long)xy[2 * u + 1] - xy[2 * v + 1];
    const long long m = dx * dx + dy * dy;
    long long k = (long long)sqrt((double)m);
    while (k * k > m) --k;
    while ((k + 1) * (k + 1) <= m) ++k;
    // m - k^2 > k  <=>  sqrt(m) > k + 1/2 (m integer: no exact halves)
    return (int32_t)(m - k * k > k ? k + 1 : k);
}

__device__ __forceinline__ int32_t arc_cost(const PrepArgs &a, int u, int v)
{
    if (a.kind == 0) return dist_coords(a.xy, u, v);
    return a.dist[(long long)u * (a.N + 1) + v];
}

// ------------------------------------------------------------------------- prep

__global__ __launch_bounds__(1024) void split_prep_kernel(PrepArgs a)
{
    __shared__ long long red[1024];
    const int tid = threadIdx.x;
    const int n = a.n;
    long long link_sum = 0;
    for (int k = tid + 1; k <= n; k += 1024) {
        const int sk = a.tour[k - 1];
        a.out.rowoff[k] = (long long)(sk - 1) * a.ld;
        if (k < n) {
            const int sn = a.tour[k];
            const int link = arc_cost(a, sk, sn);
            link_sum += link;
            a.out.w[k] = arc_cost(a, sk, 0) + arc_cost(a, 0, sn) - link;
        }
    }
    red[tid] = link_sum;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        a.out.rowoff[0] = 0;
        a.out.w[0] = arc_cost(a, 0, a.tour[0]);
        a.out.w[n] = (int32_t)(red[0] + arc_cost(a, a.tour[n - 1], 0));
        a.stats->sum = 0;
        a.stats->sq_lo = 0;
        a.stats->sq_hi = 0;
        a.stats->err_demand = 0;
        a.stats->ovf_count = 0;
    }
}

// ------------------------------------------------------------------------- lane kernel
//
// One lane = one scenario; a workgroup is one wavefront of 64 scenarios. Per lane, LDS holds
// (lane-interleaved, so any per-lane index is bank-conflict free):
//   pp  : prefix loads P_p mod 2^16 of the last 64 positions (two positions per dword),
//   suf : for the last 4 blocks of 16 positions, suffix minima of g inside each block,
//   bsf : per block b, the minimum of the block minima strictly between b and the current
//         block.
// For state i with window [s, i-1] and current block c (the block of position i-1):
//   s in an older block:  min g = min(suf[s], bsf[block(s)], running minimum of block c);
//   s in block c:         the window lies in the current block, whose g are in registers.
// The window start s advances as a two-pointer on the prefix loads (Eq. (2)); the 16-bit
// comparison is exact because every compared difference lies in [-Q, Q] and Q < 2^14.

constexpr int kLB = 16;      // positions per block
constexpr int kRing = 64;    // positions of history in LDS (4 blocks)
constexpr int kWinMax = 48;  // longest window the lane kernel answers itself

__global__ __launch_bounds__(64) void split_lane_kernel(EvalArgs a)
{
    __shared__ uint32_t pp[kRing / 2][64];
    __shared__ int32_t suf[kRing][64];
    __shared__ int32_t bsf[4][64];

    const int lane = threadIdx.x;
    const long long scen_raw = (long long)blockIdx.x * 64 + lane;
    const bool active = scen_raw < a.S;
    const long long scen = active ? scen_raw : a.S - 1;
    const uint16_t *col = a.demand + scen;
    const int64_t *rowoff = a.tour.rowoff;
    const int32_t *w = a.tour.w;
    const int n = a.n;
    const int Q = a.Q;

    uint16_t *pp16 = reinterpret_cast<uint16_t *>(&pp[0][0]);
    auto pidx = [&](int pos) { return (((pos >> 1) & (kRing / 2 - 1)) * 64 + lane) * 2 + (pos & 1); };

    pp16[pidx(0)] = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) bsf[j][lane] = kInf;

    int P = 0, s = 0, m = 0, pre = kInf;
    bool err = false, ovf = false;
    // OR of the raw 16-bit demands: bit 15 marks a negative int16 demand, which the 16-bit
    // window test cannot see (it wraps); demands in (Q, 2^15) empty the window instead.
    uint32_t qor = 0;

    uint16_t qc[kLB];
#pragma unroll
    for (int t = 0; t < kLB; ++t) qc[t] = (t + 1 <= n) ? col[rowoff[t + 1]] : (uint16_t)0;

    const int nblk = (n + kLB - 1) / kLB;
    for (int cb = 0; cb < nblk; ++cb) {
        const int cbase = cb * kLB;
        uint16_t qn[kLB];
#pragma unroll
        for (int t = 0; t < kLB; ++t) {
            const int i = cbase + kLB + t + 1;
            qn[t] = (i <= n) ? col[rowoff[i]] : (uint16_t)0;
        }
        int gb[kLB];
#pragma unroll
        for (int t = 0; t < kLB; ++t) {
            const int p = cbase + t;
            if (p >= n) continue;
            const int g = (p == 0) ? w[0] : m + w[p];
            gb[t] = g;
            pre = (t == 0) ? g : min(pre, g);
            // state i = p + 1
            const int i = p + 1;
            P += qc[t];
            qor |= qc[t];
            pp16[pidx(i)] = (uint16_t)P;
            const uint16_t T = (uint16_t)(P - Q);
            while ((int16_t)(uint16_t)(pp16[pidx(s)] - T) < 0) ++s;
            ovf |= (i - s) > kWinMax;
            if (s >= cbase) {
                err |= (s == i);
                int mm = kInf;
#pragma unroll
                for (int j = 0; j <= t; ++j)
                    if (cbase + j >= s) mm = min(mm, gb[j]);
                m = mm;
            } else {
                m = min(min(suf[s & (kRing - 1)][lane], bsf[(s >> 4) & 3][lane]), pre);
            }
        }
        if (cb + 1 < nblk) {
            int sm = gb[kLB - 1];
            suf[(cbase + kLB - 1) & (kRing - 1)][lane] = sm;
#pragma unroll
            for (int t = kLB - 2; t >= 0; --t) {
                sm = min(sm, gb[t]);
                suf[(cbase + t) & (kRing - 1)][lane] = sm;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) bsf[j][lane] = min(bsf[j][lane], sm);
            bsf[cb & 3][lane] = kInf;
        }
#pragma unroll
        for (int t = 0; t < kLB; ++t) qc[t] = qn[t];
    }

    err |= (qor & 0x8000u) != 0;
    if (active) {
        if (ovf) {
            const int k = atomicAdd(&a.stats->ovf_count, 1);
            a.ovf_list[k] = (int32_t)scen;
        } else if (err) {
            atomicOr(&a.stats->err_demand, 1);
        } else {
            a.cost[scen] = m + w[n];
        }
    }
}

// ------------------------------------------------------------------------- wave kernel

// Minimum over the 64 lanes of a wavefront with DPP row shifts and row broadcasts; the
// result is returned to every lane.
__device__ __forceinline__ int wave_min(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(kInf, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(kInf, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(kInf, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(kInf, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = min(v, __builtin_amdgcn_update_dpp(kInf, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(kInf, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// One scenario by one wavefront: the window's g values sit in LDS, lane j reads predecessor
// s + j (+ 64k for long windows), and the wavefront reduces them. Every lane runs the same
// two-pointer on the same data, so control flow stays uniform.
__device__ void wave_one(const EvalArgs &a, long long scen, int32_t *G, int32_t *PP)
{
    const int lane = threadIdx.x;
    const int n = a.n;
    const int Q = a.Q;
    const uint16_t *col = a.demand + scen;
    G[0] = a.tour.w[0];
    PP[0] = 0;
    int P = 0, s = 0;
    bool err = false;
    for (int i = 1; i <= n; ++i) {
        P += col[a.tour.rowoff[i]];
        PP[i] = P;
        while (P - PP[s] > Q) ++s;
        if (s == i) {
            err = true;
            break;
        }
        int mn = kInf;
        for (int base = s; base < i; base += 64) {
            const int p = base + lane;
            if (p < i) mn = min(mn, G[p]);
        }
        G[i] = wave_min(mn) + a.tour.w[i];
    }
    if (lane == 0) {
        if (err)
            atomicOr(&a.stats->err_demand, 1);
        else
            a.cost[scen] = G[n];
    }
    __syncthreads();
}

// mode 0: scenario k for k = blockIdx.x, blockIdx.x + gridDim.x, ... < S.
// mode 1: the scenarios queued by the lane kernel.
__global__ __launch_bounds__(64) void split_wave_kernel(EvalArgs a, int mode)
{
    extern __shared__ int32_t lds[];
    int32_t *G = lds;
    int32_t *PP = lds + (a.n + 1);
    const long long count = mode == 0 ? a.S : (long long)a.stats->ovf_count;
    for (long long k = blockIdx.x; k < count; k += gridDim.x) {
        const long long scen = mode == 0 ? k : (long long)a.ovf_list[k];
        wave_one(a, scen, G, PP);
    }
}

// ------------------------------------------------------------------------- moments

__device__ __forceinline__ void add128(unsigned long long &lo, unsigned long long &hi,
                                       unsigned long long xlo, unsigned long long xhi)
{
    const unsigned long long t = lo + xlo;
    hi += xhi + (t < lo ? 1ull : 0ull);
    lo = t;
}

__device__ void block_reduce3(unsigned long long &s, unsigned long long &lo,
                              unsigned long long &hi)
{
    __shared__ unsigned long long rs[256], rl[256], rh[256];
    const int t = threadIdx.x;
    rs[t] = s;
    rl[t] = lo;
    rh[t] = hi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            rs[t] += rs[t + off];
            unsigned long long l = rl[t], h = rh[t];
            add128(l, h, rl[t + off], rh[t + off]);
            rl[t] = l;
            rh[t] = h;
        }
        __syncthreads();
    }
    s = rs[0];
    lo = rl[0];
    hi = rh[0];
}

__global__ __launch_bounds__(256) void split_moments_partial(MomentArgs a)
{
    unsigned long long s = 0, lo = 0, hi = 0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < a.S;
         k += (long long)gridDim.x * 256) {
        const unsigned long long c = (unsigned int)a.cost[k];
        s += c;
        add128(lo, hi, c * c, 0);
    }
    block_reduce3(s, lo, hi);
    if (threadIdx.x == 0) {
        a.partials[3 * blockIdx.x + 0] = s;
        a.partials[3 * blockIdx.x + 1] = lo;
        a.partials[3 * blockIdx.x + 2] = hi;
    }
}

__global__ __launch_bounds__(256) void split_moments_final(MomentArgs a)
{
    unsigned long long s = 0, lo = 0, hi = 0;
    for (int b = threadIdx.x; b < a.nblocks; b += 256) {
        s += a.partials[3 * b + 0];
        add128(lo, hi, a.partials[3 * b + 1], a.partials[3 * b + 2]);
    }
    block_reduce3(s, lo, hi);
    if (threadIdx.x == 0) {
        a.stats->sum = s;
        a.stats->sq_lo = lo;
        a.stats->sq_hi = hi;
    }
}

// ------------------------------------------------------------------------- launchers

hipError_t launch_prep(const PrepArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(split_prep_kernel, dim3(1), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_lane(const EvalArgs &a, hipStream_t stream)
{
    const long long nb = (a.S + 63) / 64;
    hipLaunchKernelGGL(split_lane_kernel, dim3((unsigned)nb), dim3(64), 0, stream, a);
    return hipGetLastError();
}

static size_t wave_lds_bytes(int n) { return sizeof(int32_t) * 2 * ((size_t)n + 1); }

hipError_t launch_wave_all(const EvalArgs &a, hipStream_t stream)
{
    const long long nb = a.S < 65536 ? a.S : 65536;
    hipLaunchKernelGGL(split_wave_kernel, dim3((unsigned)nb), dim3(64), wave_lds_bytes(a.n),
                       stream, a, 0);
    return hipGetLastError();
}

hipError_t launch_wave_fallback(const EvalArgs &a, hipStream_t stream)
{
    const long long nb = a.S < 2048 ? a.S : 2048;
    hipLaunchKernelGGL(split_wave_kernel, dim3((unsigned)nb), dim3(64), wave_lds_bytes(a.n),
                       stream, a, 1);
    return hipGetLastError();
}

int32_t moment_blocks(int64_t S)
{
    long long b = (S + 2047) / 2048;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int32_t)b;
}

hipError_t launch_moments(const MomentArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(split_moments_partial, dim3(a.nblocks), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_moments_final, dim3(1), dim3(256), 0, stream, a);
    return hipGetLastError();
}

const char *lane_kernel_name() { return "split_lane_kernel"; }
const char *wave_kernel_name() { return "split_wave_kernel"; }

}  // namespace splitgpu
