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
        a.out.rowoff[k] = (long long)(sk - 1) * a.ld * (long long)sizeof(uint16_t);
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
    // positions n+1 .. n+kRowPad read row 0 (valid memory): lets kernels load whole blocks
    for (int k = n + 1 + tid; k <= n + kRowPad; k += 1024) a.out.rowoff[k] = 0;
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
// One lane = one scenario; a workgroup is one wavefront of 64 scenarios. Positions are
// processed in blocks of kLB = 16. Per lane, LDS holds (lane-interleaved, so a per-lane
// index costs at most a two-way bank conflict):
//   pp  : prefix loads P_p mod 2^16 of the last 64 positions, positions (2k, 2k+1) in dword k;
//         the first kMirror dwords are repeated after the ring so a 6-dword read never wraps;
//   dl  : for the last 4 blocks, the suffix minimum of g inside the block, stored as a 16-bit
//         offset from the block's minimum;
//   rec : per block b of the last 4, (minimum of g over b, minimum of the block minima
//         strictly between b and the current block).
// For state i with window [s, i-1] whose newest position i-1 lies in block c:
//   s in an older block b:  min g = min(bm[b] + dl[s], between[b], running minimum of c),
//   s in block c:           the window lies in block c, whose g values are in registers.
// Window starts (Eq. (2)) come from the prefix loads: s_i = s_{i-1} + #{p >= s_{i-1} :
// P_p < P_i - Q}. The count compares 8 (or 12) positions at once as packed 16-bit
// differences; it is exact because every compared difference lies in [-Q - q_i, Q] with
// Q < 2^14 and q_i < 2^15 (bit 15 of a demand is checked separately). Lanes whose last
// looked-ahead position expired too, or whose lookahead reached past the written prefixes,
// redo the block one position at a time. Scenarios whose windows outgrow the 64-position
// history, or whose suffix-minimum offsets outgrow 16 bits, are queued for the general kernel.
// A window start s is carried as S = (s << 7) | (lane << 1), which makes the dl offset, the
// pp row and the even base below s one instruction each.

constexpr int kLB = 16;            // positions per block
constexpr int kRingPairs = 32;     // ring of 64 positions, two per dword
constexpr int kMirror = 5;         // dwords mirrored after the ring
constexpr int kStartWinMax = 46;   // longest window at a block start the lane kernel keeps

struct LaneLds {
    uint32_t pp[kRingPairs + kMirror][64];
    uint16_t dl[4 * kLB][64];
    int32_t rec[4][64][2];
};

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) volatile uint16_t lds_u16v;
typedef __attribute__((address_space(3))) int32_t lds_i32;
typedef __attribute__((address_space(3))) char lds_char;

__device__ __forceinline__ int s_of(int S) { return S >> 7; }
__device__ __forceinline__ int S_of(int s, int lane) { return (s << 7) | (lane << 1); }

__device__ __forceinline__ uint32_t lds_dl_at(LaneLds &L, int S)
{
    return *(lds_u16 *)((lds_char *)(&L.dl[0][0]) + (S & 0x1FFE));
}
// (block minimum, between-block minimum) of the block holding s
__device__ __forceinline__ void lds_rec_at(LaneLds &L, int S, uint32_t lane8, int &bm, int &bs)
{
    const lds_i32 *r = (const lds_i32 *)((lds_char *)(&L.rec[0][0][0]) +
                                         (((uint32_t)(S >> 2) & 0x600u) | lane8));
    bm = r[0];
    bs = r[1];
}
// byte offset of pp row (s >> 1) & 31 for this lane
__device__ __forceinline__ uint32_t pp_row_off(int S, uint32_t lane4)
{
    return ((uint32_t)S & 0x1F00u) | lane4;
}
__device__ __forceinline__ uint32_t lds_pp_at(LaneLds &L, uint32_t off, int row)
{
    return *(lds_u32 *)((lds_char *)(&L.pp[0][0]) + off + row * 256);
}

// Packed 16-bit a - t in both halves (no borrow between the halves).
__device__ __forceinline__ uint32_t pk_sub16(uint32_t a, uint32_t t)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    const u16x2 av = __builtin_bit_cast(u16x2, a);
    const u16x2 tv = {(unsigned short)t, (unsigned short)t};
    return __builtin_bit_cast(uint32_t, av - tv);
}

// Bytes 0..3 = 0xFF where the matching 16-bit half of (lo.lo, lo.hi, hi.lo, hi.hi) is negative.
__device__ __forceinline__ uint32_t sign_bytes(uint32_t hi, uint32_t lo)
{
    return __builtin_amdgcn_perm(hi, lo, 0x0b0a0908u);
}

// Window start after counting expired positions from the even position below S_prev:
// cnt8 = 8 * (number of expired positions among those read).
__device__ __forceinline__ int start_from(int S_prev, uint32_t cnt8)
{
    return (int)(cnt8 << 4) + (S_prev & ~0x80);
}

// 16-bit stores, one per position: kept unmerged so no instruction packs two positions.
__device__ __forceinline__ void pp_write(LaneLds &L, int lane, int pos, uint32_t P)
{
    lds_u16v *h = (lds_u16v *)(&L.pp[0][0]);
    const int pr = (pos >> 1) & (kRingPairs - 1);
    h[(pr * 64 + lane) * 2 + (pos & 1)] = (uint16_t)P;
    if (pr < kMirror) h[((pr + kRingPairs) * 64 + lane) * 2 + (pos & 1)] = (uint16_t)P;
}

__device__ __forceinline__ bool pp_expired(LaneLds &L, int lane, int pos, uint32_t T)
{
    const uint16_t *h = reinterpret_cast<const uint16_t *>(&L.pp[0][0]);
    const int pr = (pos >> 1) & (kRingPairs - 1);
    return (int16_t)(uint16_t)(h[(pr * 64 + lane) * 2 + (pos & 1)] - (uint16_t)T) < 0;
}

// Prefix loads of the states first .. first + 15 into the ring and Pt.
template <bool kFull>
__device__ __forceinline__ void lane_prefix(LaneLds &L, int lane, int first, int n,
                                            const uint32_t (&q)[kLB], int &P, uint32_t &qor,
                                            int (&Pt)[kLB])
{
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
        if (!kFull && first + t > n) continue;
        P += q[t];
        qor |= q[t];
        Pt[t] = P;
        pp_write(L, lane, first + t, (uint32_t)P);
    }
}

// Exact one-position-at-a-time window starts for states first .. last (the rare path).
__device__ __forceinline__ void lane_starts_exact(LaneLds &L, int lane, int first, int last,
                                                  int Q, int S_start, const int (&Pt)[kLB],
                                                  int (&sA)[kLB])
{
    int s = s_of(S_start);
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
        if (first + t > last) continue;
        const uint32_t T = (uint32_t)(Pt[t] - Q);
        while (pp_expired(L, lane, s, T)) ++s;
        sA[t] = S_of(s, lane);
    }
}

// Window starts of the states 16*blk + 1 .. 16*blk + 16 (those <= n), one state at a time
// with an 8-position lookahead. Used for the first and the last block.
// In: S = start of state 16*blk. Out: sA[t] = start of state 16*blk + t + 1; S = the last.
template <bool kFull>
__device__ __forceinline__ void lane_phase_a_impl(LaneLds &L, int lane, int blk, int n, int Q,
                                                  const uint32_t (&q)[kLB], int &P, int &S,
                                                  uint32_t &qor, int (&sA)[kLB], bool &ovf)
{
    const int first = blk * kLB + 1;
    const int last = kFull ? first + kLB - 1 : min(first + kLB - 1, n);
    ovf |= S < ((first - 1 - kStartWinMax) << 7);
    int Pt[kLB];
    lane_prefix<kFull>(L, lane, first, n, q, P, qor, Pt);
    uint32_t sat = 0;
    int last_S = S;
    const uint32_t lane4 = (uint32_t)lane << 2;
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
        if (!kFull && first + t > n) continue;
        const int prev = (t == 0) ? S : sA[t - 1];
        const uint32_t T = (uint32_t)(Pt[t] - Q);
        const uint32_t off = pp_row_off(prev, lane4);
        const uint32_t d0 = lds_pp_at(L, off, 0), d1 = lds_pp_at(L, off, 1);
        const uint32_t d2 = lds_pp_at(L, off, 2), d3 = lds_pp_at(L, off, 3);
        const uint32_t m01 = sign_bytes(pk_sub16(d1, T), pk_sub16(d0, T));
        const uint32_t m23 = sign_bytes(pk_sub16(d3, T), pk_sub16(d2, T));
        sA[t] = start_from(prev, __builtin_popcount(m23) + __builtin_popcount(m01));
        sat |= m23;
        last_S = prev;
    }
    const bool rare = (int32_t)sat < 0 || (s_of(last_S) & ~1) > last - 7;
    if (rare && !ovf) lane_starts_exact(L, lane, first, last, Q, S, Pt, sA);
    S = sA[last - first];
}

__device__ __forceinline__ void lane_phase_a(LaneLds &L, int lane, int blk, int n, int Q,
                                             const uint32_t (&q)[kLB], int &P, int &S,
                                             uint32_t &qor, int (&sA)[kLB], bool &ovf)
{
    if ((blk + 1) * kLB <= n)
        lane_phase_a_impl<true>(L, lane, blk, n, Q, q, P, S, qor, sA, ovf);
    else
        lane_phase_a_impl<false>(L, lane, blk, n, Q, q, P, S, qor, sA, ovf);
}

// Window starts of two consecutive states from one read of 12 positions starting at the
// even position below the previous state's start: state t0 counts 8 of them, t1 all 12.
__device__ __forceinline__ void lane_pair_starts(LaneLds &L, uint32_t lane4, int S_prev,
                                                 uint32_t T0, uint32_t T1, int &o0, int &o1,
                                                 uint32_t &sat)
{
    const uint32_t off = pp_row_off(S_prev, lane4);
    const uint32_t d0 = lds_pp_at(L, off, 0), d1 = lds_pp_at(L, off, 1), d2 = lds_pp_at(L, off, 2);
    const uint32_t d3 = lds_pp_at(L, off, 3), d4 = lds_pp_at(L, off, 4), d5 = lds_pp_at(L, off, 5);
    const uint32_t a01 = sign_bytes(pk_sub16(d1, T0), pk_sub16(d0, T0));
    const uint32_t a23 = sign_bytes(pk_sub16(d3, T0), pk_sub16(d2, T0));
    o0 = start_from(S_prev, __builtin_popcount(a23) + __builtin_popcount(a01));
    const uint32_t b01 = sign_bytes(pk_sub16(d1, T1), pk_sub16(d0, T1));
    const uint32_t b23 = sign_bytes(pk_sub16(d3, T1), pk_sub16(d2, T1));
    const uint32_t b45 = sign_bytes(pk_sub16(d5, T1), pk_sub16(d4, T1));
    o1 = start_from(S_prev, __builtin_popcount(b45) + (__builtin_popcount(b23) +
                                                        __builtin_popcount(b01)));
    sat |= a23 | b45;  // sign bit: t0's 8th or t1's 12th position expired too
}

// Minimum of g over [s, start of block c) plus the running minimum of block c.
__device__ __forceinline__ int lane_query(LaneLds &L, int S, uint32_t lane8, int pre)
{
    int bm, bs;
    lds_rec_at(L, S, lane8, bm, bs);
    return min(min(bm + (int)lds_dl_at(L, S), bs), pre);
}

// DP of the positions p = 16*blk .. 16*blk + 15 (< n): g_p from the previous state's window
// minimum m, then the window minimum of state p + 1 into m. This careful form also handles
// windows inside the block, the empty window (q > Q) and the partial last block.
__device__ __forceinline__ void lane_phase_b(LaneLds &L, int lane, int blk, int n,
                                             const int32_t *__restrict__ w, const int (&sA)[kLB],
                                             int &m, int &pre, int (&gb)[kLB], bool &err)
{
    const int p0 = blk * kLB;
    const uint32_t lane8 = (uint32_t)lane << 3;
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
        const int p = p0 + t;
        if (p >= n) continue;
        const int g = (p == 0) ? w[0] : m + w[p];
        gb[t] = g;
        pre = (t == 0) ? g : min(pre, g);
        const int s = s_of(sA[t]);
        if (s >= p0) {
            err |= (s == p + 1);
            int mm = kInf;
#pragma unroll
            for (int j = 0; j <= t; ++j)
                if (p0 + j >= s) mm = min(mm, gb[j]);
            m = mm;
        } else {
            m = lane_query(L, sA[t], lane8, pre);
        }
    }
}

// Block blk complete: suffix minima as 16-bit offsets from the block minimum, the block's
// record, and the between-block minima of the older blocks. A scenario whose offsets do not
// fit 16 bits goes to the general kernel.
__device__ __forceinline__ void lane_block_end(LaneLds &L, int lane, int blk, const int (&gb)[kLB],
                                               bool &ovf)
{
    const int p0 = blk * kLB;
    int sm[kLB];
    sm[kLB - 1] = gb[kLB - 1];
#pragma unroll
    for (int t = kLB - 2; t >= 0; --t) sm[t] = min(sm[t + 1], gb[t]);
    const int bm = sm[0];
    ovf |= (unsigned)(sm[kLB - 1] - bm) > 0xFFFFu;  // the largest offset is the last one
#pragma unroll
    for (int t = 0; t < kLB; ++t) L.dl[(p0 + t) & (4 * kLB - 1)][lane] = (uint16_t)(sm[t] - bm);
#pragma unroll
    for (int j = 0; j < 4; ++j) L.rec[j][lane][1] = min(L.rec[j][lane][1], bm);
    L.rec[blk & 3][lane][0] = bm;
    L.rec[blk & 3][lane][1] = kInf;
}

// The common step, in one straight-line block so that the chain of LDS reads behind the
// window starts of block blk + 1 overlaps the DP arithmetic of block blk. Requires blocks
// blk and blk + 1 complete and every window of block blk to start in an older block.
__device__ __forceinline__ void lane_fast_step(LaneLds &L, int lane, int blk, int Q,
                                               const int32_t *__restrict__ w,
                                               const uint32_t (&qUse)[kLB], const int (&sCur)[kLB],
                                               int (&sNext)[kLB], int &P, int &S, uint32_t &qor,
                                               int &m, int &pre, bool &ovf)
{
    const int p0 = blk * kLB;
    const int first = p0 + kLB + 1;  // states of block blk + 1
    const uint32_t lane4 = (uint32_t)lane << 2, lane8 = (uint32_t)lane << 3;
    ovf |= S < ((first - 1 - kStartWinMax) << 7);
    int Pt[kLB];
    lane_prefix<true>(L, lane, first, first + kLB, qUse, P, qor, Pt);
    int v1[kLB], v2[kLB];
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
        int bm, bs;
        lds_rec_at(L, sCur[t], lane8, bm, bs);
        v1[t] = bm + (int)lds_dl_at(L, sCur[t]);
        v2[t] = bs;
    }
    uint32_t sat = 0;
    int gb[kLB];
    const int S_start = S;
#pragma unroll
    for (int u = 0; u < kLB / 2; ++u) {
        const int prev = (u == 0) ? S_start : sNext[2 * u - 1];
        lane_pair_starts(L, lane4, prev, (uint32_t)(Pt[2 * u] - Q), (uint32_t)(Pt[2 * u + 1] - Q),
                         sNext[2 * u], sNext[2 * u + 1], sat);
#pragma unroll
        for (int t = 2 * u; t < 2 * u + 2; ++t) {
            const int g = m + w[p0 + t];
            gb[t] = g;
            pre = (t == 0) ? g : min(pre, g);
            m = min(min(v1[t], v2[t]), pre);
        }
    }
    lane_block_end(L, lane, blk, gb, ovf);
    const int last = first + kLB - 1;
    const bool rare = (int32_t)sat < 0 || (s_of(sNext[kLB - 2]) & ~1) > last - 11;
    if (rare && !ovf) lane_starts_exact(L, lane, first, last, Q, S_start, Pt, sNext);
    S = sNext[kLB - 1];
}

// Demands of the states of block blk, by buffer loads: the descriptor holds the demand base,
// the row's byte offset is the scalar offset and the lane's scenario offset the vector one,
// so no vector instruction goes into addressing. Needs N * ld * 2 < 2^32 (host-checked).
__device__ __forceinline__ void lane_load_block(__amdgpu_buffer_rsrc_t rsrc,
                                                const int64_t *__restrict__ rowoff,
                                                uint32_t lane_off, int blk, uint32_t (&q)[kLB])
{
    // rowoff is padded past n with a valid row, so the last block loads unguarded too
#pragma unroll
    for (int t = 0; t < kLB; ++t)
        q[t] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, lane_off, (int)rowoff[blk * kLB + t + 1], 0);
}

// One block step: demands of block blk + 2, window starts of block blk + 1, DP of block blk.
__device__ __forceinline__ void lane_step(LaneLds &L, int lane, int blk, int nblk, int n, int Q,
                                          __amdgpu_buffer_rsrc_t dem,
                                          const int64_t *__restrict__ rowoff, uint32_t lane_off,
                                          const int32_t *__restrict__ w, uint32_t (&qUse)[kLB],
                                          uint32_t (&qLoad)[kLB], const int (&sCur)[kLB],
                                          int (&sNext)[kLB], int &P, int &S, uint32_t &qor,
                                          int &m, int &pre, bool &err, bool &ovf)
{
    // unconditional (rows past n are padding): keeps the load queue's wait counts exact
    lane_load_block(dem, rowoff, lane_off, blk + 2, qLoad);
    const int p0 = blk * kLB;
    const bool fast = (blk + 2) * kLB <= n && !__any(sCur[kLB - 1] >= (p0 << 7));
    if (fast) {
        lane_fast_step(L, lane, blk, Q, w, qUse, sCur, sNext, P, S, qor, m, pre, ovf);
        return;
    }
    if (blk + 1 < nblk) lane_phase_a(L, lane, blk + 1, n, Q, qUse, P, S, qor, sNext, ovf);
    int gb[kLB];
    lane_phase_b(L, lane, blk, n, w, sCur, m, pre, gb, err);
    if (blk + 1 < nblk) lane_block_end(L, lane, blk, gb, ovf);
}

// rowoff[i] here is the BYTE offset of position i's demand row.
__global__ __launch_bounds__(64) void split_lane_kernel(
    const char *__restrict__ dem_ptr, const int64_t *__restrict__ rowoff,
    const int32_t *__restrict__ w, int32_t *__restrict__ cost, DevStats *__restrict__ stats,
    int32_t *__restrict__ ovf_list, long long nscen, int n, int Q)
{
    __shared__ LaneLds L;
    const int lane = threadIdx.x;
    const long long scen_raw = (long long)blockIdx.x * 64 + lane;
    const bool active = scen_raw < nscen;
    const long long scen = active ? scen_raw : nscen - 1;
    const uint32_t lane_off = (uint32_t)scen * 2u;
    // raw buffer over the whole demand matrix (gfx9 descriptor word 3: 0x00020000)
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)dem_ptr, (short)0, -1, 0x00020000);

    pp_write(L, lane, 0, 0u);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        L.rec[j][lane][0] = kInf;
        L.rec[j][lane][1] = kInf;
    }

    int P = 0, S = S_of(0, lane), m = 0, pre = kInf;
    bool err = false, ovf = false;
    // OR of the raw 16-bit demands: bit 15 marks a negative int16 demand, which the 16-bit
    // window test cannot see (it wraps); demands in (Q, 2^15) empty the window instead.
    uint32_t qor = 0;

    const int nblk = (n + kLB - 1) / kLB;
    uint32_t q0[kLB], q1[kLB];
    int s0[kLB], s1[kLB];
    lane_load_block(rsrc, rowoff, lane_off, 0, q0);
    lane_load_block(rsrc, rowoff, lane_off, 1, q1);
    lane_phase_a(L, lane, 0, n, Q, q0, P, S, qor, s0, ovf);
    // blocks alternate the roles of (q0, q1) and (s0, s1); the loop body has no conditional
    // step so the compiler's load-wait counts stay exact across iterations
    int blk = 0;
    for (; blk + 1 < nblk; blk += 2) {
        lane_step(L, lane, blk, nblk, n, Q, rsrc, rowoff, lane_off, w, q1, q0, s0, s1, P, S, qor,
                  m, pre, err, ovf);
        lane_step(L, lane, blk + 1, nblk, n, Q, rsrc, rowoff, lane_off, w, q0, q1, s1, s0, P, S,
                  qor, m, pre, err, ovf);
    }
    if (blk < nblk)
        lane_step(L, lane, blk, nblk, n, Q, rsrc, rowoff, lane_off, w, q1, q0, s0, s1, P, S, qor,
                  m, pre, err, ovf);

    err |= (qor & 0x8000u) != 0;
    if (active) {
        if (ovf) {
            const int k = atomicAdd(&stats->ovf_count, 1);
            ovf_list[k] = (int32_t)scen;
        } else if (err) {
            atomicOr(&stats->err_demand, 1);
        } else {
            cost[scen] = m + w[n];
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

// Exclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_exclusive_sum(int v)
{
    const int lane = threadIdx.x;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    return inc - v;
}

// One scenario by one wavefront. First the prefix loads P_0..P_n are built in LDS with all
// lanes loading demands in parallel (chunk per lane + wavefront scan). Then, state by state,
// every lane runs the same two-pointer on the same data (uniform control flow), lane j reads
// g of predecessor s + j (+ 64k for long windows) and the wavefront reduces them.
__device__ void wave_one(const EvalArgs &a, long long scen, int32_t *G, int32_t *PP)
{
    const int lane = threadIdx.x;
    const int n = a.n;
    const int Q = a.Q;
    const char *dem = reinterpret_cast<const char *>(a.demand + scen);
    const int chunk = (n + 63) / 64;
    const int lo = lane * chunk + 1;
    const int hi = min(lo + chunk - 1, n);
    int local = 0;
    for (int i = lo; i <= hi; ++i) local += *(const uint16_t *)(dem + a.tour.rowoff[i]);
    int run = wave_exclusive_sum(local);
    for (int i = lo; i <= hi; ++i) {
        run += *(const uint16_t *)(dem + a.tour.rowoff[i]);
        PP[i] = run;
    }
    if (lane == 0) {
        PP[0] = 0;
        G[0] = a.tour.w[0];
    }
    __syncthreads();
    int s = 0;
    bool err = false;
    for (int i = 1; i <= n; ++i) {
        const int P = PP[i];
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
    hipLaunchKernelGGL(split_lane_kernel, dim3((unsigned)nb), dim3(64), 0, stream,
                       reinterpret_cast<const char *>(a.demand), a.tour.rowoff, a.tour.w, a.cost,
                       a.stats, a.ovf_list, (long long)a.S, a.n, a.Q);
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
