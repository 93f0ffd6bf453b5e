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

#include <mutex>

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

// One workgroup per tour: the weights w, the row offsets and the padding of tour t, and the
// zeroed result block of the tour. Workgroup 0 also resets the batch counters. Workgroups
// past the call's T return at once.
__global__ __launch_bounds__(1024) void split_prep_kernel(PrepArgs a)
{
    __shared__ long long red[16];
    __shared__ int32_t ends[2];  // c(0, first customer), c(last customer, 0)
    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    if (t >= *a.tour.nt) return;
    const int32_t *tour = a.tour.tours + a.tour.tptr[t];
    const int n = (int)(a.tour.tptr[t + 1] - a.tour.tptr[t]);
    const int64_t ab = tour_abase(a.tour.tptr, t);
    int64_t *rowoff = a.tour.rowoff + ab;
    uint32_t *rowoff32 = a.tour.rowoff32 + ab;
    int32_t *w = a.tour.w + ab;
    long long link_sum = 0;
    for (int k = tid + 1; k <= n; k += 1024) {
        const int sk = tour[k - 1];
        rowoff[k] = (long long)(sk - 1) * a.ld * (long long)sizeof(uint16_t);
        rowoff32[k] = (uint32_t)rowoff[k];
        // the two depot arcs of w_0 and w_n, from the threads that hold their customers
        if (k == 1) ends[0] = arc_cost(a, 0, sk);
        if (k == n) ends[1] = arc_cost(a, sk, 0);
        if (k < n) {
            const int sn = tour[k];
            const int link = arc_cost(a, sk, sn);
            link_sum += link;
            w[k] = arc_cost(a, sk, 0) + arc_cost(a, 0, sn) - link;
        }
    }
    // sum of the links: within each wavefront, then over the 16 wavefronts (integers: the
    // order does not change the result)
    for (int off = 32; off > 0; off >>= 1) link_sum += __shfl_xor(link_sum, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = link_sum;
    __syncthreads();
    if (tid == 0) {
        for (int i = 1; i < 16; ++i) red[0] += red[i];
    }
    // positions n+1 .. n+kRowPad: row 0 (valid memory), absent for the lane kernel, weight 0,
    // so that kernels can load whole blocks of positions past n without guards
    for (int k = n + 1 + tid; k <= n + kRowPad; k += 1024) {
        rowoff[k] = 0;
        rowoff32[k] = kRowAbsent;
        w[k] = 0;
    }
    if (tid == 0) {
        rowoff[0] = 0;
        rowoff32[0] = kRowAbsent;
        w[0] = ends[0];
        w[n] = (int32_t)(red[0] + ends[1]);
        DevStats *st = a.stats + t;
        st->sum = 0;
        st->sq_lo = 0;
        st->sq_hi = 0;
        st->err_demand = 0;
        st->ovf_count = 0;
        if (t == 0) {
            a.ctl->head = 0;
            a.ctl->ovf_total = 0;
        }
    }
}

// ------------------------------------------------------------------------- lane kernel
//
// One lane = one scenario; a workgroup is one wavefront of 64 scenarios. States 0..n are
// processed in blocks of LB states (block c = states LB*c .. LB*c + LB-1), LB = 16 or 8, a
// launch choice. A block's windows may reach back over the three blocks before it (windows
// of up to 3 * LB - 1 positions always fit): 16-state blocks suit windows of about 16 to 47
// positions; shorter windows mostly start inside a 16-state block, which takes the slow
// state-by-state path, and 8-state blocks keep them in older blocks. For state i, Eq. (3)'s
// window is [s_i, i-1] with s_i = #{p : P_p < P_i - Q} (Eq. (2); P = prefix loads).
//
// LDS per wavefront, every array interleaved by lane:
//   rec : per block slot c & 3, the pair (minimum of g over block c, minimum of the block
//         minima strictly between block c and the block being evaluated);
//   dl  : suffix minima of g inside each block of the last 64 positions, as 16-bit offsets
//         from the block minimum (row = position & 63);
//   pp  : prefix loads P mod 2^16 of the last 64 positions, positions (2k, 2k+1) in dword row
//         k & 31; rows 0 .. kMirror-1 repeated after the ring so that an 8-row read never wraps.
// The window minimum of a state of block c whose window starts at s in an older block b is
//   min(rec[b].bm + dl[s], rec[b].bs, minimum of g over block c before the state).
// Window starts advance by counting expired positions as packed 16-bit differences: the two
// states of a pair share one read of 12 positions starting at the even position below the
// previous start; in a fast block the first counts 8 of them and the second 10 (12 elsewhere).
// A block where some lane's last counted position expired (the count may be short), or where a
// count reached past the written prefix loads, has its starts redone. The counts are exact while
// 8 * max(q) + Q < 2^15 (every compared difference then fits a signed 16-bit value).
// Scenarios the kernel cannot finish exactly (that demand bound broken, a window longer than
// its history, suffix offsets beyond 16 bits) are queued for the general kernel.
//
// A window start s is carried as S = (s << 7) | (lane << 1): the dl offset, the pp row, the
// rec slot and the even base below s take one or two instructions each. The block loop is
// unrolled 64 / LB times so that every LDS store has a constant offset.

constexpr int kRingPairs = 32;  // prefix-load ring of 64 positions, two per dword
constexpr int kMirror = 7;      // ring rows repeated after the ring

// Blocks of LB states: kSteps = blocks in the 64-position history (the unroll of the block
// loop), kLog = log2(LB). The ring, the suffix offsets and the four block records hold every
// window start of a block that lies at most three blocks back, so 4 * LB <= 64.
template <int LB>
struct LaneCfg {
    static_assert(LB == 16 || LB == 8, "blocks of 16 or 8 states");
    static constexpr int kSteps = 64 / LB;
    static constexpr int kLog = LB == 16 ? 4 : 3;
};

struct __attribute__((aligned(16))) LaneLds {
    uint64_t rec[4][64];
    uint16_t dl[64][64];
    uint32_t pp[kRingPairs + kMirror][64];
};
constexpr uint32_t kRecOff = 0;
constexpr uint32_t kDlOff = sizeof(uint64_t) * 4 * 64;
constexpr uint32_t kPpOff = kDlOff + sizeof(uint16_t) * 64 * 64;

// Read-only per-tour arrays (written by the prep kernel, a previous launch): the constant
// address space lets every uniform read of them be a scalar load.
typedef __attribute__((address_space(4))) const uint32_t cu32;
typedef __attribute__((address_space(4))) const int32_t ci32;
typedef __attribute__((address_space(4))) const int64_t ci64;

typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) char lds_char;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int s_of(int S) { return S >> 7; }
__device__ __forceinline__ int S_of(int s, int lane) { return (s << 7) | (lane << 1); }

__device__ __forceinline__ const lds_char *lds_base(LaneLds &L)
{
    return (const lds_char *)(&L);
}

// Window-minimum lookup of a start S (in an older block): the 16-bit suffix offset and the
// block record; combined later by query_min so that the reads are in flight meanwhile.
// The record slot (s / LB) & 3, 512 bytes a slot, is bits 9..10 of S >> (log2(LB) - 2).
template <int LB>
__device__ __forceinline__ void query_issue(LaneLds &L, int S, uint32_t lane8, uint32_t &dlv,
                                            uint64_t &recv)
{
    constexpr int kSh = LaneCfg<LB>::kLog - 2;
    dlv = *(const lds_u16 *)(lds_base(L) + kDlOff + ((uint32_t)S & 0x1FFEu));
    recv = *(const lds_u64 *)(lds_base(L) + kRecOff + ((((uint32_t)S >> kSh) & 0x600u) | lane8));
}
__device__ __forceinline__ int query_min(uint32_t dlv, uint64_t recv, int pre)
{
    const int bm = (int)(uint32_t)recv;
    const int bs = (int)(uint32_t)(recv >> 32);
    return min(min(bm + (int)dlv, bs), pre);
}

__device__ __forceinline__ uint32_t pp_at(LaneLds &L, uint32_t off, int row)
{
    return *(const lds_u32 *)(lds_base(L) + kPpOff + off + row * 256);
}
// 16-bit ring value of position p
__device__ __forceinline__ uint32_t pp_pos(LaneLds &L, int lane, int p)
{
    const lds_u16 *h = (const lds_u16 *)(lds_base(L) + kPpOff);
    return h[(((p >> 1) & (kRingPairs - 1)) * 64 + lane) * 2 + (p & 1)];
}

// Packed 16-bit a - t in both halves, t a 16-bit value (no borrow between the halves).
__device__ __forceinline__ uint32_t pk_sub16(uint32_t a, uint32_t t)
{
    const u16x2 av = __builtin_bit_cast(u16x2, a);
    const u16x2 tv = {(unsigned short)t, (unsigned short)t};
    return __builtin_bit_cast(uint32_t, av - tv);
}
// Bytes 0..3 = 0xFF where the matching 16-bit half of (lo.lo, lo.hi, hi.lo, hi.hi) is negative.
__device__ __forceinline__ uint32_t sign_bytes(uint32_t hi, uint32_t lo)
{
    return __builtin_amdgcn_perm(hi, lo, 0x0b0a0908u);
}

// Exact start of a state with threshold T, advancing one position at a time from a start that
// is not past it. Bounded: position i of the state is never expired, and the ring holds it.
__device__ __forceinline__ int exact_start(LaneLds &L, int lane, int S, uint32_t T)
{
    int s = s_of(S);
    for (int k = 0; k < 2 * kRingPairs; ++k) {
        if ((int16_t)(uint16_t)(pp_pos(L, lane, s) - T) >= 0) break;
        ++s;
    }
    return S_of(s, lane);
}

// Prefix loads of block c (R = c mod 64/LB): q[j] is the demand of position LB*c + j (zero
// where a position does not exist). Writes the ring rows of the block and returns the packed
// thresholds TT[k] = (P_{LB*c+2k} - Q, P_{LB*c+2k+1} - Q) mod 2^16.
template <int LB, int R>
__device__ __forceinline__ void lane_prefix(LaneLds &L, int lane, const uint16_t (&q)[LB],
                                            uint32_t QQ, uint32_t &Plast, uint32_t &qor,
                                            uint32_t (&TT)[LB / 2])
{
    uint32_t prev = Plast;
#pragma unroll
    for (int k = 0; k < LB / 2; ++k) {
        // (q0, q1) packed by one byte permutation, then (q0, q0 + q1): the low half shifted
        // into the high half adds q0 there and leaves the low half alone
        const u16x2 qv = {q[2 * k], q[2 * k + 1]};
        const uint32_t Qp = __builtin_bit_cast(uint32_t, qv);
        const uint32_t E = Qp + (Qp << 16);
        const u16x2 ev = __builtin_bit_cast(u16x2, E);
        const u16x2 pv = __builtin_bit_cast(u16x2, prev);
        const u16x2 bc = {pv.y, pv.y};
        const uint32_t PP = __builtin_bit_cast(uint32_t, ev + bc);
        prev = PP;
        TT[k] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, PP) -
                                                 __builtin_bit_cast(u16x2, QQ));
        qor |= Qp;  // both halves: the bound below takes the larger
        constexpr int row0 = (LB / 2) * R;
        L.pp[(row0 + k) & (kRingPairs - 1)][lane] = PP;
        if (((row0 + k) & (kRingPairs - 1)) < kMirror)
            L.pp[((row0 + k) & (kRingPairs - 1)) + kRingPairs][lane] = PP;
    }
    Plast = prev;
}

template <int LB>
__device__ __forceinline__ uint32_t tt_half(const uint32_t (&TT)[LB / 2], int t)
{
    return (t & 1) ? (TT[t >> 1] >> 16) : (TT[t >> 1] & 0xFFFFu);
}

// Window starts of the states first .. first + LB-1, one state at a time with an 8-position
// lookahead, completed exactly where the lookahead saturated or reached past the last written
// prefix load (first + LB-1). States past n (demand 0) get valid starts too. In: Sp = start of
// state first - 1.
template <int LB>
__device__ __forceinline__ void lane_starts_careful(LaneLds &L, int lane, int first,
                                                    const uint32_t (&TT)[LB / 2], int Sp,
                                                    int (&sOut)[LB])
{
    const uint32_t lane4 = (uint32_t)lane << 2;
#pragma unroll
    for (int t = 0; t < LB; ++t) {
        const uint32_t T = tt_half<LB>(TT, t);
        const uint32_t off = ((uint32_t)Sp & 0x1F00u) | lane4;
        const uint32_t d0 = pp_at(L, off, 0), d1 = pp_at(L, off, 1);
        const uint32_t d2 = pp_at(L, off, 2), d3 = pp_at(L, off, 3);
        const uint32_t a01 = sign_bytes(pk_sub16(d1, T), pk_sub16(d0, T));
        const uint32_t a23 = sign_bytes(pk_sub16(d3, T), pk_sub16(d2, T));
        const int base = Sp & ~0x80;
        int Sn = base + (int)((__builtin_popcount(a23) + __builtin_popcount(a01)) << 4);
        // A short count (the eighth position expired too) is exact up to its end: every counted
        // position expired, so the walk continues from there. A read past the written prefix
        // loads (first + LB-1) may have counted stale positions: the walk starts over from Sp.
        const bool past = s_of(base) + 7 > first + LB - 1;
        const bool redo = (int32_t)a23 < 0 || past;
        if (redo) Sn = exact_start(L, lane, past ? Sp : Sn, T);
        sOut[t] = Sn;
        Sp = Sn;
    }
}

// Materializes v at this point of the instruction stream (keeps the compiler from sinking a
// computation towards a later use).
__device__ __forceinline__ void pin(int &v) { asm volatile("" : "+v"(v)); }

// The 12 positions a pair reads (6 packed dwords) and the even position they start at.
struct PairData {
    uint32_t d[6];
    int base;
};
__device__ __forceinline__ PairData pair_read(LaneLds &L, uint32_t lane4, int Sp)
{
    PairData p;
    const uint32_t off = ((uint32_t)Sp & 0x1F00u) | lane4;
#pragma unroll
    for (int r = 0; r < 6; ++r) p.d[r] = pp_at(L, off, r);
    p.base = Sp & ~0x80;
    return p;
}
// Start of a state with threshold T counted over the first 2 * D positions of a pair's read;
// last < 0: the last counted position expired too (the count may be short).
template <int D>
__device__ __forceinline__ int pair_count(const PairData &p, uint32_t T, uint32_t &last)
{
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < D; r += 2) {
        const uint32_t x = sign_bytes(pk_sub16(p.d[r + 1], T), pk_sub16(p.d[r], T));
        cnt = __builtin_popcount(x) + cnt;
        last = x;
    }
    return p.base + (int)(cnt << 4);
}

// Start counted over the first 10 positions of a pair's read; last < 0: position 9 expired.
__device__ __forceinline__ int pair_count10(const PairData &p, uint32_t T, uint32_t &last)
{
    const uint32_t x0 = sign_bytes(pk_sub16(p.d[1], T), pk_sub16(p.d[0], T));
    const uint32_t x1 = sign_bytes(pk_sub16(p.d[3], T), pk_sub16(p.d[2], T));
    const uint32_t x2 = sign_bytes(pk_sub16(p.d[4], T), 0u);
    last = x2;
    uint32_t cnt = __builtin_popcount(x0);
    cnt = __builtin_popcount(x1) + cnt;
    cnt = __builtin_popcount(x2) + cnt;
    return p.base + (int)(cnt << 4);
}

// Window starts of the states first .. first + LB-1 from Sp (start of state first - 1) with the
// pair counts; where a count may be short or a read reached past the written prefix loads
// (first + LB-1), the block is redone state by state.
template <int LB>
__device__ __forceinline__ void lane_starts_pairs(LaneLds &L, int lane, int first,
                                                  const uint32_t (&TT)[LB / 2], int Sp,
                                                  int (&sOut)[LB])
{
    const uint32_t lane4 = (uint32_t)lane << 2;
    const int S_in = Sp;
    uint32_t sat = 0;
#pragma unroll
    for (int u = 0; u < LB / 2; ++u) {
        const PairData p = pair_read(L, lane4, Sp);
        uint32_t x0, x1;
        sOut[2 * u] = pair_count<4>(p, TT[u] & 0xFFFFu, x0);
        sOut[2 * u + 1] = pair_count<6>(p, TT[u] >> 16, x1);
        sat |= x0 | x1;
        Sp = sOut[2 * u + 1];
    }
    if (__any((int32_t)sat < 0 || (s_of(sOut[LB - 3]) & ~1) > first + LB - 12))
        lane_starts_careful<LB>(L, lane, first, TT, S_in, sOut);
}

// 16 positions (8 packed dwords) from the even position below Sp.
struct WideData {
    uint32_t d[8];
    int base;
};
__device__ __forceinline__ WideData wide_read(LaneLds &L, uint32_t lane4, int Sp)
{
    WideData p;
    const uint32_t off = ((uint32_t)Sp & 0x1F00u) | lane4;
#pragma unroll
    for (int r = 0; r < 8; ++r) p.d[r] = pp_at(L, off, r);
    p.base = Sp & ~0x80;
    return p;
}
template <int D>
__device__ __forceinline__ int wide_count(const WideData &p, uint32_t T, uint32_t &last)
{
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < D; r += 2) {
        const uint32_t x = sign_bytes(pk_sub16(p.d[r + 1], T), pk_sub16(p.d[r], T));
        cnt = __builtin_popcount(x) + cnt;
        last = x;
    }
    return p.base + (int)(cnt << 4);
}
// Redo of a block's starts after the fast counts fell short or read past the written prefix
// loads: pairs again, from one 16-position read each, the first state counting 12 positions and
// the second all 16 (half the serial reads of a state-by-state redo, which has no other work
// left to overlap); where those fall short or read past the written prefix loads too, state by
// state. Used for 16-state blocks (an 8-state block's ring rarely holds 16 positions ahead).
template <int LB>
__device__ __forceinline__ void lane_starts_wide(LaneLds &L, int lane, int first,
                                                 const uint32_t (&TT)[LB / 2], int Sp,
                                                 int (&sOut)[LB])
{
    const uint32_t lane4 = (uint32_t)lane << 2;
    const int S_in = Sp;
    uint32_t sat = 0;
#pragma unroll
    for (int u = 0; u < LB / 2; ++u) {
        const WideData p = wide_read(L, lane4, Sp);
        uint32_t x0, x1;
        sOut[2 * u] = wide_count<6>(p, TT[u] & 0xFFFFu, x0);
        sOut[2 * u + 1] = wide_count<8>(p, TT[u] >> 16, x1);
        sat |= x0 | x1;
        Sp = sOut[2 * u + 1];
    }
    if (__any((int32_t)sat < 0 || (s_of(sOut[LB - 3]) & ~1) > first + LB - 16))
        lane_starts_careful<LB>(L, lane, first, TT, S_in, sOut);
}

// g of state t of a block (t uniform). Written as explicit selects: the compiler would
// otherwise turn it into an indexed load from a scratch copy of the whole block.
template <int LB>
__device__ __forceinline__ int block_g_at(const int (&gb)[LB], int t)
{
    t = __builtin_amdgcn_readfirstlane(t);
    int g = gb[0];
#pragma unroll
    for (int k = 1; k < LB; ++k) {
        int m = __builtin_amdgcn_readfirstlane(-(int)(t == k));
        asm volatile("" : "+s"(m));  // an opaque 0 / -1 mask
        g = (gb[k] & m) | (g & ~m);
    }
    return g;
}

// Block c complete (R = c mod 64/LB): suffix minima as 16-bit offsets from the block minimum,
// and the records of blocks c, c-1, c-2 (bm1, bm2: minima of blocks c-1, c-2).
template <int LB, int R>
__device__ __forceinline__ void lane_block_end(LaneLds &L, int lane, const int (&gb)[LB],
                                               int &bm1, int &bm2, bool &ovf)
{
    int sm[LB];
    sm[LB - 1] = gb[LB - 1];
#pragma unroll
    for (int t = LB - 2; t >= 0; --t) sm[t] = min(sm[t + 1], gb[t]);
    const int bm = sm[0];
    ovf |= (unsigned)(sm[LB - 1] - bm) > 0xFFFFu;  // the largest offset is the last one
#pragma unroll
    for (int t = 0; t < LB; ++t) L.dl[LB * R + t][lane] = (uint16_t)(sm[t] - bm);
    auto pack = [](int lo, int hi) {
        return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
    };
    L.rec[R & 3][lane] = pack(bm, kInf);
    L.rec[(R + 3) & 3][lane] = pack(bm1, bm);
    L.rec[(R + 2) & 3][lane] = pack(bm2, min(bm, bm1));
    bm2 = bm1;
    bm1 = bm;
}

// DP of block c, state by state, for any window position (inside the block, or empty).
// States past n (demand 0, weight 0) are evaluated too and not used.
template <int LB>
__device__ __forceinline__ void lane_dp_careful(LaneLds &L, int lane, int c,
                                                ci32 *__restrict__ w,
                                                const int (&sCur)[LB], int (&gb)[LB], bool &err)
{
    const int p0 = c * LB;
    const uint32_t lane8 = (uint32_t)lane << 3;
    // every state's older-block lookup, issued up front (in bounds for any start; a lane whose
    // window lies inside the block does not use its result)
    uint32_t qd[LB];
    uint64_t qr[LB];
#pragma unroll
    for (int t = 0; t < LB; ++t) query_issue<LB>(L, sCur[t], lane8, qd[t], qr[t]);
    int pre = kInf;
#pragma unroll
    for (int t = 0; t < LB; ++t) {
        const int i = p0 + t;
        int g;
        if (i == 0) {
            g = w[0];
        } else {
            const int s = s_of(sCur[t]);
            int m;
            if (s >= p0) {  // window inside the block, or empty (s == i: q_i > Q)
                err |= (s >= i);
                int mm = kInf;
                if (s == p0) {
                    mm = pre;  // the whole block so far (block 0 of a long-window tour)
                } else {
#pragma unroll
                    for (int j = 0; j < t; ++j)
                        if (p0 + j >= s) mm = min(mm, gb[j]);
                }
                m = mm;
            } else {
                m = query_min(qd[t], qr[t], pre);
            }
            g = w[i] + m;
        }
        gb[t] = g;
        pre = min(pre, g);
    }
}

// Demands of block blk, by buffer loads: the descriptor holds the demand base, the row's byte
// offset is the scalar offset and the lane's scenario offset the vector one. rowoff is padded
// past n with a valid row, so blocks past n load unguarded (their values are not used).
template <int LB>
__device__ __forceinline__ void lane_load_block(__amdgpu_buffer_rsrc_t rsrc,
                                                cu32 *__restrict__ rowoff,
                                                uint32_t lane_off, int blk, uint16_t (&q)[LB])
{
#pragma unroll
    for (int t = 0; t < LB; ++t)
        q[t] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, lane_off, (int)rowoff[blk * LB + t], 0);
}

// The LB weights of block blk by vector loads (every lane the same 16 bytes, LB / 4 times): a
// scalar load here would need a wait that also drains every outstanding LDS operation.
typedef int i32x4 __attribute__((ext_vector_type(4)));
template <int LB>
__device__ __forceinline__ void lane_load_w(__amdgpu_buffer_rsrc_t wrsrc, int blk, int (&wv)[LB])
{
#pragma unroll
    for (int j = 0; j < LB / 4; ++j) {
        const i32x4 v = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                       wrsrc, 0, (blk * LB + 4 * j) * 4, 0));
        wv[4 * j] = v.x;
        wv[4 * j + 1] = v.y;
        wv[4 * j + 2] = v.z;
        wv[4 * j + 3] = v.w;
    }
}

struct LaneState {
    uint32_t Plast;  // high half: prefix load of the last position written to the ring
    uint32_t qor;    // OR of the demands read
    int bm1, bm2;    // minima of the last two completed blocks
    int gres;        // g_n
    bool err, ovf;
};

// One block step (R = c mod 64/LB): demands of block c + 3, window starts of block c + 1, DP
// of block c. qUse holds the demands of block c + 1, qLoad receives those of block c + 3.
template <int LB, int R>
__device__ __forceinline__ void lane_step(LaneLds &L, int lane, int c, int n, uint32_t QQ,
                                          __amdgpu_buffer_rsrc_t dem, __amdgpu_buffer_rsrc_t wrsrc,
                                          cu32 *__restrict__ rowoff, uint32_t lane_off,
                                          ci32 *__restrict__ w, const uint16_t (&qUse)[LB],
                                          uint16_t (&qLoad)[LB], const int (&sCur)[LB],
                                          int (&sNext)[LB], const int (&wUse)[LB],
                                          int (&wLoad)[LB], LaneState &st)
{
    // weights of block c + 1 (used by the next step), demands of block c + 3; unconditional,
    // so that every path has the same vector-memory wait counts
    lane_load_w<LB>(wrsrc, c + 1, wLoad);
    lane_load_block<LB>(dem, rowoff, lane_off, c + 3, qLoad);
    const int nb = n >> LaneCfg<LB>::kLog;
    if (c > nb) return;
    const int p0 = c * LB;
    const int first = p0 + LB;  // states of block c + 1
    const uint32_t lane4 = (uint32_t)lane << 2, lane8 = (uint32_t)lane << 3;
    // the ring and the block records must still hold every window start of block c + 1
    // (state LB*c + LB-1 exists whenever block c + 1 does)
    if (c + 1 <= nb) st.ovf |= sCur[LB - 1] < ((p0 - 2 * LB) << 7);
    int gb[LB];
    // states past n (demand 0, weight 0) are evaluated like the others and not used
    const bool fast = c >= 1 && !__any(sCur[LB - 1] >= (p0 << 7));
    if (fast) {
        // Software pipeline over the LB/2 pairs of block c + 1 and the LB states of block c.
        // Iteration u: window lookups for the DP of the next pair, DP of states 2u, 2u+1,
        // first state of pair u-1, then second state of pair u (whose read was issued at the
        // end of iteration u-1) and the read of pair u+1. The scheduling barriers keep the
        // independent work between each read and its first use.
        // the block's weights, in vector registers since the previous step
        int wv[LB];
#pragma unroll
        for (int t = 0; t < LB; ++t) wv[t] = wUse[t];
        uint32_t TT[LB / 2];
        lane_prefix<LB, (R + 1) % LaneCfg<LB>::kSteps>(L, lane, qUse, QQ, st.Plast, st.qor, TT);
        uint32_t qd[LB];
        uint64_t qr[LB];
        query_issue<LB>(L, sCur[0], lane8, qd[0], qr[0]);
        query_issue<LB>(L, sCur[1], lane8, qd[1], qr[1]);
        PairData pcur = pair_read(L, lane4, sCur[LB - 1]);
        PairData pprev = pcur;
        uint32_t sat = 0;  // sign bit: some count of this lane may be short
        int pre = kInf;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < LB / 2; ++u) {
            if (u + 1 < LB / 2) {
                query_issue<LB>(L, sCur[2 * u + 2], lane8, qd[2 * u + 2], qr[2 * u + 2]);
                query_issue<LB>(L, sCur[2 * u + 3], lane8, qd[2 * u + 3], qr[2 * u + 3]);
            }
#pragma unroll
            for (int t = 2 * u; t < 2 * u + 2; ++t) {
                const int g = wv[t] + query_min(qd[t], qr[t], pre);
                gb[t] = g;
                pre = min(pre, g);
            }
            if (u > 0) {
                uint32_t x;
                sNext[2 * u - 2] = pair_count<4>(pprev, TT[u - 1] & 0xFFFFu, x);
                sat |= x;
                pin(sNext[2 * u - 2]);
            }
            __builtin_amdgcn_sched_barrier(0);
            uint32_t x1;
            sNext[2 * u + 1] = pair_count10(pcur, TT[u] >> 16, x1);
            sat |= x1;
            pprev = pcur;
            if (u + 1 < LB / 2) pcur = pair_read(L, lane4, sNext[2 * u + 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        {
            uint32_t x;
            sNext[LB - 2] = pair_count<4>(pprev, TT[LB / 2 - 1] & 0xFFFFu, x);
            sat |= x;
        }
        // no later block reads the last block's records (and its suffix offsets would hold
        // g_n = f_n, which need not fit 16 bits)
        if (c < nb) lane_block_end<LB, R>(L, lane, gb, st.bm1, st.bm2, st.ovf);
        // the last pair counts positions up to its base + 9; the ring is written up to
        // first + LB-1. Either condition below is rare: redo the block's starts (16-state
        // blocks with wider pair counts first, then state by state where those fall short).
        if (__any((int32_t)sat < 0 || (s_of(sNext[LB - 3]) & ~1) > first + LB - 10)) {
            if constexpr (LB == 16)
                lane_starts_wide<LB>(L, lane, first, TT, sCur[LB - 1], sNext);
            else
                lane_starts_careful<LB>(L, lane, first, TT, sCur[LB - 1], sNext);
        }
        if (c == nb) st.gres = block_g_at<LB>(gb, n & (LB - 1));
        return;
    }
    // careful step (positions past n load demand 0)
    if (c + 1 <= nb) {
        uint32_t TT[LB / 2];
        lane_prefix<LB, (R + 1) % LaneCfg<LB>::kSteps>(L, lane, qUse, QQ, st.Plast, st.qor, TT);
        lane_starts_pairs<LB>(L, lane, first, TT, sCur[LB - 1], sNext);
    }
    lane_dp_careful<LB>(L, lane, c, w, sCur, gb, st.err);
    if (c + 1 <= nb) {
        lane_block_end<LB, R>(L, lane, gb, st.bm1, st.bm2, st.ovf);
    } else {
        st.gres = block_g_at<LB>(gb, n & (LB - 1));  // block c holds state n
    }
}

// Issue priority by progress through the work item: 3 over the first quarter of its blocks,
// down to 0 over the last. Among waves of equal priority a SIMD issues from the oldest, which
// drives the items of its two wavefronts half an item apart, so that at the end of a launch one
// of them runs alone for about half an item. Favouring the wavefront that is less far along
// keeps the two in step (measured on one tour: the two last items of a SIMD end about 14 us
// apart instead of 57, and the launch takes about 1% less). Used only when every item has the
// same length (one tour, or tours of one length): in a batch of uneven tours the items' ends
// are spread anyway, and this order measured about 0.5-0.9% slower there.
__device__ __forceinline__ void item_priority(int c, int nb)
{
    const int x = 4 * c, m = nb + 1;
    if (x < m)
        __builtin_amdgcn_s_setprio(3);
    else if (x < 2 * m)
        __builtin_amdgcn_s_setprio(2);
    else if (x < 3 * m)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// One work item: the 64 scenarios sb*64 .. sb*64+63 of tour t.
template <int LB>
__device__ __forceinline__ void lane_item(LaneLds &L, const EvalArgs &a, int t, long long sb,
                                          __amdgpu_buffer_rsrc_t rsrc, bool by_progress)
{
    const int lane = threadIdx.x;
    const long long nscen = a.S;
    // tour values come from memory: state that they are the same on every lane
    ci64 *tptr = (ci64 *)a.tour.tptr;
    const int64_t p0 = tptr[t];
    const int n = (int)(tptr[t + 1] - p0);
    const int64_t ab = p0 + (int64_t)t * (1 + kRowPad);
    cu32 *__restrict__ rowoff = (cu32 *)a.tour.rowoff32 + ab;
    ci32 *__restrict__ w = (ci32 *)a.tour.w + ab;
    const long long scen_raw = sb * 64 + lane;
    const bool active = scen_raw < nscen;
    const long long scen = active ? scen_raw : nscen - 1;
    const uint32_t lane_off = (uint32_t)scen * 2u;
    const int Q = a.Q;
    const uint32_t QQ = (uint32_t)Q | ((uint32_t)Q << 16);

    LaneState st;
    st.Plast = 0;
    st.qor = 0;
    st.bm1 = kInf;
    st.bm2 = kInf;
    st.gres = 0;
    st.err = false;
    st.ovf = false;

    const int nb = n >> LaneCfg<LB>::kLog;
    uint16_t qA[LB], qB[LB], qC[LB], qD[LB];
    int sA[LB], sB[LB];
    int wA[LB], wB[LB];  // weights of the block a step evaluates, loaded one step ahead
    const __amdgpu_buffer_rsrc_t wrsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.tour.w + ab), (short)0, (int)(sizeof(int32_t) * (n + 1 + kRowPad)), 0x00020000);
#pragma unroll
    for (int k = 0; k < LB; ++k) {
        sA[k] = S_of(0, lane);
        sB[k] = S_of(0, lane);
    }
    lane_load_w<LB>(wrsrc, 0, wA);
    lane_load_block<LB>(rsrc, rowoff, lane_off, 0, qA);
    lane_load_block<LB>(rsrc, rowoff, lane_off, 1, qB);
    lane_load_block<LB>(rsrc, rowoff, lane_off, 2, qC);
    {
        // block 0: position 0 has no demand (P_0 = 0, its row offset is absent); start 0
        uint32_t TT[LB / 2];
        lane_prefix<LB, 0>(L, lane, qA, QQ, st.Plast, st.qor, TT);
        lane_starts_pairs<LB>(L, lane, 0, TT, S_of(0, lane), sA);
    }
    // block b's demands live in q[A, B, C, D][b & 3], its starts and weights in [A, B][b & 1];
    // 64 / LB steps per iteration keep these roles and the LDS rows of every step constant
    for (int c = 0; c <= nb; c += LaneCfg<LB>::kSteps) {
        if (by_progress) item_priority(c, nb);
        lane_step<LB, 0>(L, lane, c, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qB, qD, sA, sB, wA, wB, st);
        lane_step<LB, 1>(L, lane, c + 1, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qC, qA, sB, sA, wB, wA, st);
        lane_step<LB, 2>(L, lane, c + 2, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qD, qB, sA, sB, wA, wB, st);
        lane_step<LB, 3>(L, lane, c + 3, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qA, qC, sB, sA, wB, wA, st);
        if constexpr (LaneCfg<LB>::kSteps == 8) {
            lane_step<LB, 4>(L, lane, c + 4, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qB, qD, sA, sB, wA, wB, st);
            lane_step<LB, 5>(L, lane, c + 5, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qC, qA, sB, sA, wB, wA, st);
            lane_step<LB, 6>(L, lane, c + 6, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qD, qB, sA, sB, wA, wB, st);
            lane_step<LB, 7>(L, lane, c + 7, n, QQ, rsrc, wrsrc, rowoff, lane_off, w, qA, qC, sB, sA, wB, wA, st);
        }
    }

    __builtin_amdgcn_s_setprio(0);
    // counts exact only while 8 * max(q) + Q < 2^15 (qor >= max(q)); bit 15 (a negative
    // int16 demand) also lands here, and the general kernel reports it
    st.ovf |= 8u * ((st.qor | (st.qor >> 16)) & 0xFFFFu) + (uint32_t)Q > 32767u;
    int32_t *cost = a.cost + (long long)t * a.ldc;
    if (active) {
        if (st.ovf) {
            cost[scen] = kCostOvf;
            atomicAdd(&a.stats[t].ovf_count, 1);
            atomicAdd(&a.ctl->ovf_total, 1u);
        } else if (st.err) {
            atomicOr(&a.stats[t].err_demand, 1);
        } else {
            cost[scen] = st.gres;
        }
    }
}

// Work item k = (tour order[k / nsb], scenario block k % nsb), nsb = ceil(S / 64). Workgroup b
// runs item b, then either items b + gridDim.x, b + 2 gridDim.x, ... (lane_static) or items
// gridDim.x, gridDim.x + 1, ... taken from a queue until none is left (a grid of at least
// T * nsb workgroups runs one item each). A queue index is fetched while the current item runs.
template <int LB>
__global__ __launch_bounds__(64) void split_lane_kernel(EvalArgs a)
{
    __shared__ LaneLds L;
    const int lane = threadIdx.x;
    // raw buffer over the demand bytes the tours can address (gfx9 descriptor word 3:
    // 0x00020000); loads at offsets past lane_bytes (absent positions) return 0
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)a.demand, (short)0, (int)a.lane_bytes, 0x00020000);
    const long long nsb = (a.S + 63) / 64;
    const long long items = nsb * *(ci64 *)a.tour.nt;
    const bool queue = (long long)gridDim.x < items;
    uint32_t k = blockIdx.x;
    while ((long long)k < items) {
        uint32_t knext = 0xFFFFFFFFu;
        if (queue) {
            if (a.lane_static)
                knext = k + gridDim.x;
            else if (lane == 0)
                knext = gridDim.x + atomicAdd(&a.ctl->head, 1u);
        }
        const long long r = (long long)k / nsb;
        const int t = ((ci32 *)a.tour.order)[r];
        lane_item<LB>(L, a, t, (long long)k - r * nsb, rsrc, a.lane_uniform != 0);
        k = __builtin_amdgcn_readfirstlane(knext);
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
__device__ void wave_one(const EvalArgs &a, int t, long long scen, int32_t *G, int32_t *PP)
{
    const int lane = threadIdx.x;
    const int64_t ab = tour_abase(a.tour.tptr, t);
    const int n = (int)(a.tour.tptr[t + 1] - a.tour.tptr[t]);
    const int64_t *rowoff = a.tour.rowoff + ab;
    const int32_t *w = a.tour.w + ab;
    const int Q = a.Q;
    const char *dem = reinterpret_cast<const char *>(a.demand + scen);
    const int chunk = (n + 63) / 64;
    const int lo = lane * chunk + 1;
    const int hi = min(lo + chunk - 1, n);
    int local = 0;
    uint32_t qor = 0;
    for (int i = lo; i <= hi; ++i) {
        const uint32_t q = *(const uint16_t *)(dem + rowoff[i]);
        local += (int)q;
        qor |= q;
    }
    // a negative int16 demand (bit 15) is rejected for any Q, also where Q admits 2^15 and more
    const bool neg = __any((qor & 0x8000u) != 0);
    int run = wave_exclusive_sum(local);
    for (int i = lo; i <= hi; ++i) {
        run += *(const uint16_t *)(dem + rowoff[i]);
        PP[i] = run;
    }
    if (lane == 0) {
        PP[0] = 0;
        G[0] = w[0];
    }
    __syncthreads();
    int s = 0;
    bool err = neg;
    for (int i = 1; i <= n && !err; ++i) {
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
        G[i] = wave_min(mn) + w[i];
    }
    if (lane == 0) {
        if (err)
            atomicOr(&a.stats[t].err_demand, 1);
        else
            a.cost[(long long)t * a.ldc + scen] = G[n];
    }
    __syncthreads();
}

// mode 0: every (tour, scenario) pair, k = t * S + s over k = blockIdx.x, blockIdx.x +
//         gridDim.x, ...
// mode 1: the pairs the lane kernel marked kCostOvf; a workgroup scans 64 costs of one tour
//         at a time and evaluates the marked ones. Returns at once when nothing was marked.
__global__ __launch_bounds__(64) void split_wave_kernel(EvalArgs a, int mode)
{
    extern __shared__ int32_t lds[];
    int32_t *G = lds;
    int32_t *PP = lds + (a.maxn + 1);
    const long long T = *a.tour.nt;
    if (mode == 0) {
        for (long long k = blockIdx.x; k < T * a.S; k += gridDim.x) {
            const int t = (int)(k / a.S);
            wave_one(a, t, k - (long long)t * a.S, G, PP);
        }
        return;
    }
    if (a.ctl->ovf_total == 0) return;
    const long long nsb = (a.S + 63) / 64;
    for (long long k = blockIdx.x; k < T * nsb; k += gridDim.x) {
        const int t = (int)(k / nsb);
        const long long s0 = (k - (long long)t * nsb) * 64;
        const long long scen = s0 + threadIdx.x;
        const bool marked = scen < a.S && a.cost[(long long)t * a.ldc + scen] == kCostOvf;
        unsigned long long m = __ballot(marked);
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            wave_one(a, t, s0 + j, G, PP);
        }
    }
}

// ------------------------------------------------------------------------- two-kernel form

// The paper's literal two-kernel form, kept as an ablation of the fused lane kernel: first the
// Eq. (2) window starts of every (state, scenario) are written to an int16 matrix in HBM
// (row abase(t) + i, scenario fastest), then a second kernel reads them back and takes each
// window's minimum by scanning it.

// One lane per scenario of work item (tour, 64-scenario block): prefix loads with a two-pointer;
// mask = smallest p with P_i - P_p <= Q (p == i when q_i > Q: the window is empty).
__global__ __launch_bounds__(64) void split_mask_kernel(EvalArgs a, int16_t *mask,
                                                        long long mask_ld)
{
    const long long nsb = (a.S + 63) / 64;
    const long long k = blockIdx.x;
    const long long T = *a.tour.nt;
    if (k >= nsb * T) return;
    const int t = (int)(k / nsb);
    const long long scen = (k - (long long)t * nsb) * 64 + threadIdx.x;
    if (scen >= a.S) return;
    const int64_t ab = tour_abase(a.tour.tptr, t);
    const int n = (int)(a.tour.tptr[t + 1] - a.tour.tptr[t]);
    const int64_t *rowoff = a.tour.rowoff + ab;
    const char *dem = reinterpret_cast<const char *>(a.demand + scen);
    int P = 0, Ps = 0, s = 0;
    for (int i = 1; i <= n; ++i) {
        const uint32_t q = *(const uint16_t *)(dem + rowoff[i]);
        P += (int)q;
        while (s < i && P - Ps > a.Q) {
            ++s;
            Ps += *(const uint16_t *)(dem + rowoff[s]);
        }
        // a negative int16 demand (bit 15) gets an empty window: reported as infeasible
        mask[(ab + i) * mask_ld + scen] = (int16_t)((q & 0x8000u) ? i : s);
    }
}

// One lane per scenario: g_i = w_i + min of g over [mask_i, i - 1], scanning the window in a
// 64-entry history of g per lane in LDS. A window longer than 63 states sends the scenario to
// the general kernel (cost marked kCostOvf); an empty window reports an infeasible demand.
__global__ __launch_bounds__(64) void split_masked_dp_kernel(EvalArgs a, const int16_t *mask,
                                                             long long mask_ld)
{
    __shared__ int ring[64][64];
    const int lane = threadIdx.x;
    const long long nsb = (a.S + 63) / 64;
    const long long k = blockIdx.x;
    const long long T = *a.tour.nt;
    if (k >= nsb * T) return;
    const int t = (int)(k / nsb);
    const long long scen_raw = (k - (long long)t * nsb) * 64 + lane;
    const bool active = scen_raw < a.S;
    const long long scen = active ? scen_raw : a.S - 1;
    const int64_t ab = tour_abase(a.tour.tptr, t);
    const int n = (int)(a.tour.tptr[t + 1] - a.tour.tptr[t]);
    const int32_t *w = a.tour.w + ab;
    bool err = false, ovf = false;
    int g = w[0];
    ring[0][lane] = g;
    for (int i = 1; i <= n; ++i) {
        int s = mask[(ab + i) * mask_ld + scen];
        err |= s >= i;
        ovf |= i - s > 63;
        if (s < i - 63) s = i - 63;
        // uniform trip count: the longest window of the wavefront (at most 63)
        int len = i - s;
        for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
        int m = kInf;
        for (int d = 1; d <= len; ++d) {
            const int p = i - d;
            if (p >= s) m = min(m, ring[p & 63][lane]);
        }
        g = w[i] + m;
        ring[i & 63][lane] = g;
    }
    if (!active) return;
    if (ovf) {
        a.cost[(long long)t * a.ldc + scen] = kCostOvf;
        atomicAdd(&a.stats[t].ovf_count, 1);
        atomicAdd(&a.ctl->ovf_total, 1u);
    } else if (err) {
        atomicOr(&a.stats[t].err_demand, 1);
    } else {
        a.cost[(long long)t * a.ldc + scen] = g;
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

// grid (nblocks, T_grid): workgroup (b, t) sums a strided share of tour t's costs
__global__ __launch_bounds__(256) void split_moments_partial(MomentArgs a)
{
    const int t = blockIdx.y;
    if (t >= *a.nt) return;
    const int32_t *cost = a.cost + (long long)t * a.ldc;
    unsigned long long s = 0, lo = 0, hi = 0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < a.S;
         k += (long long)gridDim.x * 256) {
        const unsigned long long c = (unsigned int)cost[k];
        s += c;
        add128(lo, hi, c * c, 0);
    }
    block_reduce3(s, lo, hi);
    if (threadIdx.x == 0) {
        unsigned long long *p = a.partials + 3 * ((long long)t * a.nblocks + blockIdx.x);
        p[0] = s;
        p[1] = lo;
        p[2] = hi;
    }
}

// grid T_grid: workgroup t combines the partials of tour t
__global__ __launch_bounds__(256) void split_moments_final(MomentArgs a)
{
    const int t = blockIdx.x;
    if (t >= *a.nt) return;
    const unsigned long long *p = a.partials + 3 * (long long)t * a.nblocks;
    unsigned long long s = 0, lo = 0, hi = 0;
    for (int b = threadIdx.x; b < a.nblocks; b += 256) {
        s += p[3 * b + 0];
        add128(lo, hi, p[3 * b + 1], p[3 * b + 2]);
    }
    block_reduce3(s, lo, hi);
    if (threadIdx.x == 0) {
        a.stats[t].sum = s;
        a.stats[t].sq_lo = lo;
        a.stats[t].sq_hi = hi;
    }
}

// ------------------------------------------------------------------------- scratch

// Fixed device scratch of the allocation-free evaluation (split_eval_noalloc): every per-call
// device buffer of a one-tour evaluation (staged tour, per-position arrays, result block,
// counters, moment partials) is carved from it. Each GPU holds its own copy for the life of the
// process; its device address is looked up once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **out)
{
    static std::mutex mu;
    static void *addr[kMaxScratchDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

// ------------------------------------------------------------------------- launchers

hipError_t launch_prep(const PrepArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(split_prep_kernel, dim3(a.tour.T_grid), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_lane(const EvalArgs &a, hipStream_t stream)
{
    if (a.lane_block == 8)
        hipLaunchKernelGGL(split_lane_kernel<8>, dim3((unsigned)a.lane_grid), dim3(64), 0, stream,
                           a);
    else
        hipLaunchKernelGGL(split_lane_kernel<16>, dim3((unsigned)a.lane_grid), dim3(64), 0,
                           stream, a);
    return hipGetLastError();
}

static size_t wave_lds_bytes(int maxn) { return sizeof(int32_t) * 2 * ((size_t)maxn + 1); }

// Dynamic LDS beyond the default 64 KiB (tours near the maximum length) must be opted into.
static hipError_t wave_lds_allow(size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)split_wave_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_wave_all(const EvalArgs &a, hipStream_t stream)
{
    hipError_t e = wave_lds_allow(wave_lds_bytes(a.maxn));
    if (e != hipSuccess) return e;
    const long long work = a.S * a.tour.T_grid;
    const long long nb = work < a.wave_grid ? work : a.wave_grid;
    hipLaunchKernelGGL(split_wave_kernel, dim3((unsigned)nb), dim3(64), wave_lds_bytes(a.maxn), stream,
                       a, 0);
    return hipGetLastError();
}

hipError_t launch_wave_fallback(const EvalArgs &a, hipStream_t stream)
{
    hipError_t e = wave_lds_allow(wave_lds_bytes(a.maxn));
    if (e != hipSuccess) return e;
    const long long work = (a.S + 63) / 64 * a.tour.T_grid;
    const long long nb = work < 2048 ? work : 2048;
    hipLaunchKernelGGL(split_wave_kernel, dim3((unsigned)nb), dim3(64), wave_lds_bytes(a.maxn), stream,
                       a, 1);
    return hipGetLastError();
}

hipError_t launch_mask(const EvalArgs &a, int16_t *mask, long long mask_ld, hipStream_t stream)
{
    const long long items = (a.S + 63) / 64 * a.tour.T_grid;
    hipLaunchKernelGGL(split_mask_kernel, dim3((unsigned)items), dim3(64), 0, stream, a, mask,
                       mask_ld);
    return hipGetLastError();
}

hipError_t launch_masked_dp(const EvalArgs &a, const int16_t *mask, long long mask_ld,
                            hipStream_t stream)
{
    const long long items = (a.S + 63) / 64 * a.tour.T_grid;
    hipLaunchKernelGGL(split_masked_dp_kernel, dim3((unsigned)items), dim3(64), 0, stream, a,
                       mask, mask_ld);
    return hipGetLastError();
}

const char *mask_kernel_name() { return "split_mask_kernel+split_masked_dp_kernel"; }

int32_t moment_blocks(int64_t S)
{
    long long b = (S + 2047) / 2048;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int32_t)b;
}

hipError_t launch_moments(const MomentArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(split_moments_partial, dim3(a.nblocks, a.T_grid), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_moments_final, dim3(a.T_grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

const char *lane_kernel_name() { return "split_lane_kernel"; }
const char *wave_kernel_name() { return "split_wave_kernel"; }

}  // namespace splitgpu
