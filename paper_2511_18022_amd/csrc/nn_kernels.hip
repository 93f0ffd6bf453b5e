// HIP kernels of the tour-encoder surrogate on gfx950: features along the tour, four 5-tap
// conv layers of width 128 as implicit GEMMs on bf16 MFMA (fp32 accumulation), mean-pool and
// MLP head, the backward pass, Adam, and a top-k selection for screening.
//
// Layout: activations are bf16 [T][n + 4][C] (position-major, channels fastest) with two zero
// rows before and after every tour. The 5-tap window of output position j is then the
// contiguous span of 5 * C values starting at padded row j, so the conv is a GEMM whose A rows
// overlap in memory (no im2col copy): out[j][co] = sum_kk X[(row j) * C + kk] * Wf[co][kk],
// kk = tap * C + ci. The backward-data conv is the same GEMM with the flipped, transposed
// weights Wb[ci][tap' * 128 + co] = W[4 - tap'][ci][co].
//
// MFMA v_mfma_f32_16x16x32_bf16 (checked on the device): lane l holds A[row l % 16][k (l/16)*8
// + e], B[k (l/16)*8 + e][col l % 16], and D[row (l/16)*4 + i][col l % 16], e < 8, i < 4.
//
// Every reduction runs in a fixed order, so results are bitwise reproducible run to run.
#include <type_traits>

#include "nn_internal.h"

namespace splitgpu {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// fp32 -> bf16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits_f32(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// fp64 -> bf16 bits, round to nearest, ties to even, directly from the double (no fp32 step)
__device__ __forceinline__ uint16_t bf16_bits_f64(double x)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned long long sign = u >> 63;
    u &= 0x7FFFFFFFFFFFFFFFull;
    if (u == 0) return (uint16_t)(sign << 15);
    // keep 7 fraction bits of the 52: round at bit 45
    const unsigned long long lsb = (u >> 45) & 1ull;
    u += 0xFFFFFFFFFFFull + lsb;  // half a unit (2^44) - 1 + lsb
    const int e = (int)(u >> 52) - 1023;  // unbiased exponent after rounding
    const uint32_t frac = (uint32_t)((u >> 45) & 0x7Fu);
    // the values here are normal and well inside the bf16 range
    const uint32_t be = (uint32_t)(e + 127);
    return (uint16_t)((sign << 15) | (be << 7) | frac);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// fp32 -> bf16 bits by the hardware conversion (round to nearest, ties to even: the same bits
// as bf16_bits_f32 for every finite value) in one instruction
__device__ __forceinline__ uint16_t bf16_bits_hw(float x)
{
    const f32x2_t v = {x, 0.f};
    return (uint16_t)__builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// ------------------------------------------------------------------------- demand statistics

// One workgroup per customer: exact integer sums of q and q^2 over the S scenarios, then the
// mean and population standard deviation in double.
__global__ __launch_bounds__(256) void nn_dstats_kernel(const int16_t *demand, int64_t ld,
                                                        int64_t S, double *musd)
{
    __shared__ long long s1[256], s2[256];
    const int c = blockIdx.x;
    const int16_t *row = demand + (long long)c * ld;
    long long a = 0, b = 0;
    for (long long s = threadIdx.x; s < S; s += 256) {
        const long long q = row[s];
        a += q;
        b += q * q;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = (double)s1[0] / (double)S;
        const double m2 = (double)s2[0] / (double)S;
        const double var = m2 - mu * mu;
        musd[2 * c] = mu;
        musd[2 * c + 1] = sqrt(var > 0.0 ? var : 0.0);
    }
}

// ------------------------------------------------------------------------- features

__device__ __forceinline__ long long nn_dist(const NnInstance &in, int u, int v)
{
    if (in.kind == 1) return in.dist[(long long)u * (in.N + 1) + v];
    const long long dx = (long long)in.xy[2 * u] - in.xy[2 * v];
    const long long dy = (long long)in.xy[2 * u + 1] - in.xy[2 * v + 1];
    const long long m = dx * dx + dy * dy;
    long long k = (long long)sqrt((double)m);
    while (k * k > m) --k;
    while ((k + 1) * (k + 1) <= m) ++k;
    return m - k * k > k ? k + 1 : k;
}

// One thread per (tour, position): the 8 features in double, rounded once to bf16, written
// with the 24 zero channels as 64 contiguous bytes. Out-of-range ids set *err and read id 1.
__global__ __launch_bounds__(256) void nn_features_kernel(NnInstance in, const int32_t *tours,
                                                          int32_t T, int32_t n,
                                                          const double *musd, int32_t Q, double L,
                                                          uint16_t *X, int32_t packed,
                                                          int32_t *err)
{
    const long long m = (long long)blockIdx.x * 256 + threadIdx.x;
    if (m >= (long long)T * n) return;
    const int t = (int)(m / n), j = (int)(m - (long long)t * n);
    const int32_t *tour = tours + (long long)t * n;
    auto id = [&](int k) {
        int c = tour[k];
        if (c < 1 || c > in.N) {
            atomicOr(err, 1);
            c = 1;
        }
        return c;
    };
    const int c = id(j);
    const int prev = j > 0 ? id(j - 1) : 0;
    const int nxt = j + 1 < n ? id(j + 1) : 0;
    double f[8];
    if (in.kind == 0) {
        f[0] = ((double)in.xy[2 * c] - (double)in.xy[0]) / L;
        f[1] = ((double)in.xy[2 * c + 1] - (double)in.xy[1]) / L;
    } else {
        f[0] = 0.0;
        f[1] = 0.0;
    }
    f[2] = musd[2 * (c - 1)] / (double)Q;
    f[3] = musd[2 * (c - 1) + 1] / (double)Q;
    f[4] = (double)nn_dist(in, prev, c) / L;
    f[5] = (double)nn_dist(in, c, nxt) / L;
    f[6] = (double)nn_dist(in, 0, c) / L;
    f[7] = 1.0;
    u16x8 v;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = bf16_bits_f64(f[k]);
    if (packed) {  // prediction input: [T][n][8], no padding rows or channels
        *reinterpret_cast<u16x8 *>(X + m * kNnFeatures) = v;
        return;
    }
    u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    u16x8 *dst = reinterpret_cast<u16x8 *>(X + ((long long)t * (n + 4) + j + 2) * kNnCi0);
    dst[0] = v;
    dst[1] = zero;
    dst[2] = zero;
    dst[3] = zero;
}

// ------------------------------------------------------------------------- conv (MFMA)

// Y[t][j + 2][co] for M = T * n positions. A workgroup is 4 wavefronts; each wavefront computes
// 64 positions x 128 channels: 4 x 8 tiles of 16 x 16, K = 5 * CI in blocks of 32. The weights
// are staged in LDS a group of GB K blocks (GB x 8 KB) at a time, double-buffered, with one
// barrier per group: the group after next is loaded into registers while a group runs. The
// activation fragments of a block are loaded kConvDepth blocks before it runs, into a register
// ring (the K loop is unrolled so that every ring slot is a fixed register set). The register
// budget (at most 256 per lane) lets two wavefronts share each SIMD, whose MFMA work then
// covers the other's waits.
// LDS holds a block as [k quarter][co] so that the 16-byte reads of the 16 lanes of a column
// group hit consecutive addresses.
// MODE 0: Y = bf16(relu(acc + bias[co]))       (forward)
// MODE 1: Y = bf16(acc) where mask > 0, else 0 (backward data: mask = the layer's input H)
// Wavefronts past the last position run the loop on a clamped row (every barrier is reached)
// and store nothing.
constexpr int kConvDepth = 2;  // K blocks of activation loads in flight

template <int CI, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void nn_conv_kernel(
    const uint16_t *__restrict__ X, const uint16_t *__restrict__ Wt, const float *__restrict__ bias,
    const uint16_t *__restrict__ mask, uint16_t *__restrict__ Y, int32_t T, int32_t n)
{
    constexpr int K = kNnTaps * CI;
    constexpr int KB = K / 32;
    constexpr int D = KB < kConvDepth ? KB : kConvDepth;
    constexpr int GB = KB % 2 == 0 ? 2 : KB;  // K blocks per staged weight group
    constexpr int NG = KB / GB;
    constexpr int BLK = 4 * kNnWidth;         // bf16x8 chunks of one K block
    __shared__ bf16x8 Bs[2][GB * BLK];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const long long M = (long long)T * n;
    const long long m0 = ((long long)blockIdx.x * 4 + wave) * 64;
    const int r16 = lane & 15, kq = lane >> 4;
    // A row starts (padded row j of tour t, tap 0) of this lane's 4 positions
    const bf16x8 *arow[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        long long m = m0 + mt * 16 + r16;
        if (m >= M) m = M - 1;  // the ragged tail reads a valid row; its result is not stored
        const long long t = m / n, j = m - t * n;
        arow[mt] = reinterpret_cast<const bf16x8 *>(X + (t * (n + 4) + j) * CI + kq * 8);
    }
    // this thread stages chunks c = tid and tid + 256 of each block: co = c & 127, k quarter
    // c >> 7, i.e. Wt[co][kb * 32 + quarter * 8 .. + 8]
    const bf16x8 *wsrc0 = reinterpret_cast<const bf16x8 *>(Wt + (long long)(tid & 127) * K +
                                                            (tid >> 7) * 8);
    const bf16x8 *wsrc1 = wsrc0 + 2;  // quarter + 2
    const int wdst0 = (tid >> 7) * kNnWidth + (tid & 127), wdst1 = wdst0 + 2 * kNnWidth;
    f32x4 acc[4][8];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // activation ring: slot q holds the fragments of blocks q, q + D, ...
    bf16x8 ra[D][4];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ra[q][mt] = arow[mt][q * 4];
    // weight group 0 to LDS; group 1 into registers
    bf16x8 wr[GB][2];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
        Bs[0][q * BLK + wdst0] = wsrc0[q * 4];
        Bs[0][q * BLK + wdst1] = wsrc1[q * 4];
    }
    if (NG > 1) {
#pragma unroll
        for (int q = 0; q < GB; ++q) {
            wr[q][0] = wsrc0[(GB + q) * 4];
            wr[q][1] = wsrc1[(GB + q) * 4];
        }
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int g = kb / GB, q = kb % GB, cur = g & 1;
        const int slot = kb % D;
        bf16x8 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = ra[slot][mt];
        // the slot's fragments are in a[]: refill it with block kb + D
        if (kb + D < KB) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) ra[slot][mt] = arow[mt][(kb + D) * 4];
        }
        bf16x8 b[8];
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) b[nt] = Bs[cur][q * BLK + kq * kNnWidth + nt * 16 + r16];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt],
                                                                      0, 0, 0);
        if (q == GB - 1 && g + 1 < NG) {
            // group g + 1 to the other buffer (last read in group g - 1, before the previous
            // barrier), group g + 2 into registers
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                Bs[cur ^ 1][u * BLK + wdst0] = wr[u][0];
                Bs[cur ^ 1][u * BLK + wdst1] = wr[u][1];
            }
            if (g + 2 < NG) {
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    wr[u][0] = wsrc0[((g + 2) * GB + u) * 4];
                    wr[u][1] = wsrc1[((g + 2) * GB + u) * 4];
                }
            }
            __syncthreads();
        }
    }
    if (m0 >= M) return;
    // D rows (lane / 16) * 4 + i of each 16-row tile, column lane % 16 of each 16-column tile.
    // Row mb + off (off <= 51) is position jb + off of tour tb, carried into the next tours
    // past their ends: one division per lane. The bias values (MODE 0) are loaded once, and a
    // tile's 32 mask values (MODE 1) are all requested before the first is used.
    const long long mb = m0 + (lane >> 4) * 4;
    const long long tb = mb / n;
    const int jb = (int)(mb - tb * n);
    float bco[8];
    if (MODE == 0) {
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) bco[nt] = bias[nt * 16 + r16];
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        long long base[4];
        bool live[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int off = mt * 16 + i;
            live[i] = mb + off < M;
            long long t = tb;
            int j = jb + off;
            while (j >= n) {
                j -= n;
                ++t;
            }
            // a row past the last position addresses row 0 (read only under MODE 1's mask,
            // never written)
            base[i] = live[i] ? (t * (n + 4) + j + 2) * kNnWidth : 0;
        }
        uint16_t mk[4][8];
        if (MODE == 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) mk[i][nt] = mask[base[i] + nt * 16 + r16];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (!live[i]) continue;
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                float v = acc[mt][nt][i];
                if (MODE == 0) {
                    v += bco[nt];
                    v = v > 0.f ? v : 0.f;
                } else {
                    if (mk[i][nt] == 0 || (mk[i][nt] & 0x8000u)) v = 0.f;
                }
                Y[base[i] + nt * 16 + r16] = bf16_bits_hw(v);
            }
        }
    }
}

// ------------------------------------------------------------------------- fused inference

// All four conv layers of one tile of kFuseTP positions of one tour in LDS, for prediction only
// (training keeps every layer's output for the backward pass). The input tile carries a halo
// of 8 rows (2 per layer); layer l's output row r is position j0 - 6 + 2l + r, and rows at
// positions outside the tour are set to zero, which is the zero padding of the next layer. Each
// layer is a GEMM over 16-row m-tiles x 128 channels: wave p owns channel pair p (tiles 2p and
// 2p + 1) over every m-tile, so each weight fragment it reads from L2 (in fragment order, 1 KB
// contiguous per tile and K block) feeds all the m-tiles of the layer. The fragments form one stream
// over the four layers, kept kFuseDepth K blocks ahead in a register ring, so a layer starts
// with its first fragments already loaded and the K loop has no barrier (one per layer). The
// input tile shares its LDS with the second hidden buffer, which is first written by layer 2,
// after every wave has passed layer 2's barrier and so finished reading the input. The last
// layer rounds its outputs to bfloat16 (as the layer-by-layer path stores them) and sums them
// per channel over the tile's positions, in a fixed order, into zpart[t][tile][co].
constexpr int kFuseTP = 128;                       // output positions per tile
constexpr int kFuseMT = (kFuseTP + 12 + 15) / 16;  // m-tiles of layers 1..3 (TP + 12, 8, 4 rows)
constexpr int kFuseRows = kFuseMT * 16 + 4;        // rows of an LDS buffer (taps read 4 past)
constexpr int kFuseDepth = 2;                      // K blocks of weight fragments in flight
constexpr int kFuseThreads = 256;                  // four waves, one per channel pair
constexpr int kFuseOcc = 2;                        // waves per SIMD the register budget allows
constexpr int kFuseK1 = 64;  // layer 1's K: 5 taps x 8 features, zero-padded to 2 blocks of 32
constexpr int kFuseStrideX = kNnCi0 + 8;    // bf16 per input row (16 bytes of padding)
constexpr int kFuseStrideH = kNnWidth + 8;  // bf16 per hidden row (16 bytes of padding)
static_assert(kFuseTP % 16 == 0, "the last layer covers the tile in whole m-tiles");
static_assert(kNnFeatures == 8 && kNnTaps * kNnFeatures <= kFuseK1,
              "a tap's features are one 16-byte fragment; the taps fit layer 1's packed K");
static_assert(kFuseDepth >= 1 && kFuseDepth <= kFuseK1 / 32,
              "the prologue fills the ring from layer 1's K blocks alone");

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two floats to bf16 bits in one instruction (round to nearest, ties to even, as
// bf16_bits_f32): lo in bits 0..15, hi in bits 16..31.
__device__ __forceinline__ uint32_t bf16x2_bits(float lo, float hi)
{
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// K of a layer with CI input channels in the fused kernel (layer 1 packs its 8 features)
__host__ __device__ constexpr int fuse_k(int ci) { return ci == kNnCi0 ? kFuseK1 : kNnTaps * ci; }

struct FuseRing {
    bf16x8 b0[kFuseDepth], b1[kFuseDepth];  // fragments of channel tiles 2p and 2p + 1
};

// Fragment kb of channel pair cp from the fragment-ordered weights Wg of a layer with K inputs.
template <int K>
__device__ __forceinline__ void fuse_frag(const uint16_t *Wg, int cp, int kb, bf16x8 &x0,
                                          bf16x8 &x1)
{
    const int lane = threadIdx.x & 63;
    const uint16_t *p = Wg + ((cp * (K / 32) + kb) * 2 * 64 + lane) * 8;
    x0 = *reinterpret_cast<const bf16x8 *>(p);
    x1 = *reinterpret_cast<const bf16x8 *>(p + 64 * 8);
}

// The MC m-tiles of one layer for channel pair cp. Fragment kb of this layer
// sits in ring slot (R0 + kb) % depth; the slot it frees is refilled with the fragment depth
// blocks later in the stream, which is in the next layer (weights Wn, CIN input channels; none
// when CIN == 0) near the end. Without POOL the outputs go to `out`; with POOL, sum[h] receives
// this lane's share of the channel sums of tile 2cp + h (its 4 rows of each m-tile).
template <int CI, int MC, int R0, int CIN, bool POOL>
__device__ __forceinline__ void fused_part(const uint16_t *in, uint16_t *out, const uint16_t *Wt,
                                           const uint16_t *Wn, const float *bias, int pos0,
                                           int n, int cp, FuseRing &ring, float (&sum)[2])
{
    constexpr int K = fuse_k(CI);
    constexpr int KB = K / 32;
    constexpr int KN = CIN ? fuse_k(CIN) : 0;
    constexpr int KBN = KN / 32;
    constexpr int D = kFuseDepth;
    constexpr int SIN = CI == kNnCi0 ? kFuseStrideX : kFuseStrideH;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    f32x4 acc[MC][2];
#pragma unroll
    for (int mt = 0; mt < MC; ++mt) acc[mt][0] = acc[mt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    // activation fragment of m-tile mt for K block kb: for layer 1, k = 8 tap + feature (taps
    // past the fifth are zero); otherwise k = CI tap + channel
    auto frag_a = [&](int kb, int mt) {
        const int kk = kb * 32 + kq * 8;
        if (CI == kNnCi0) {
            const int tap = kk / kNnFeatures;
            const int tc = tap < kNnTaps ? tap : kNnTaps - 1;
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(in + (mt * 16 + r16 + tc) * SIN);
            const bf16x8 z = {};
            return tap < kNnTaps ? v : z;
        }
        const int tap = kk / CI, ci = kk - tap * CI;
        return *reinterpret_cast<const bf16x8 *>(in + (mt * 16 + r16 + tap) * SIN + ci);
    };
    bf16x8 a[MC];
#pragma unroll
    for (int mt = 0; mt < MC; ++mt) a[mt] = frag_a(0, mt);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int slot = (R0 + kb) % D;
        const bf16x8 bb0 = ring.b0[slot], bb1 = ring.b1[slot];
        if (kb + D < KB)
            fuse_frag<K>(Wt, cp, kb + D, ring.b0[slot], ring.b1[slot]);
        else if (kb + D - KB < KBN)
            fuse_frag<KN>(Wn, cp, kb + D - KB, ring.b0[slot], ring.b1[slot]);
        // each m-tile's next fragment is read as soon as its two products are issued
#pragma unroll
        for (int mt = 0; mt < MC; ++mt) {
            acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bb0, acc[mt][0], 0, 0, 0);
            acc[mt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bb1, acc[mt][1], 0, 0, 0);
            if (kb + 1 < KB) a[mt] = frag_a(kb + 1, mt);
        }
        // keep the compiler from hoisting later blocks' reads into this one: their registers
        // would push the wave past the budget of two waves per SIMD and into scratch
        __builtin_amdgcn_sched_barrier(0);
    }
    // bias, ReLU, rows outside the tour zeroed (MASK; a layer whose rows all lie inside the
    // tour, the uniform common case, needs no row test), then bf16 two rows at a time
    auto epilogue = [&](auto mask_tag) {
        constexpr bool MASK = decltype(mask_tag)::value;
#pragma unroll
        for (int mt = 0; mt < MC; ++mt) {
            const int r0 = mt * 16 + kq * 4;  // this lane's 4 rows: r0 .. r0 + 3
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int co = (2 * cp + h) * 16 + r16;
                const float b = bias[co];
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = fmaxf(acc[mt][h][i] + b, 0.f);
                    if (MASK) {
                        const int pos = pos0 + r0 + i;
                        v[i] = pos >= 0 && pos < n ? v[i] : 0.f;
                    }
                }
                const uint32_t p01 = bf16x2_bits(v[0], v[1]), p23 = bf16x2_bits(v[2], v[3]);
                if (POOL) {
                    sum[h] += __uint_as_float(p01 << 16);
                    sum[h] += __uint_as_float(p01 & 0xFFFF0000u);
                    sum[h] += __uint_as_float(p23 << 16);
                    sum[h] += __uint_as_float(p23 & 0xFFFF0000u);
                } else {
                    uint16_t *o = out + r0 * kFuseStrideH + co;
                    o[0] = (uint16_t)p01;
                    o[kFuseStrideH] = (uint16_t)(p01 >> 16);
                    o[2 * kFuseStrideH] = (uint16_t)p23;
                    o[3 * kFuseStrideH] = (uint16_t)(p23 >> 16);
                }
            }
        }
    };
    if (pos0 >= 0 && pos0 + MC * 16 <= n)
        epilogue(std::false_type{});
    else
        epilogue(std::true_type{});
}

// One layer over MT m-tiles (see fused_part). With POOL the tile's channel sums go to
// pool_out[128].
template <int CI, int MT, int R0, int CIN, bool POOL>
__device__ __forceinline__ void fused_layer(const uint16_t *in, uint16_t *out,
                                            const uint16_t *Wt, const uint16_t *Wn,
                                            const float *bias, int pos0, int n, float *pool_out,
                                            FuseRing &ring)
{
    const int cp = threadIdx.x >> 6;
    float sum[2] = {0.f, 0.f};
    __syncthreads();  // the input rows of this layer are in LDS
    fused_part<CI, MT, R0, CIN, POOL>(in, out, Wt, Wn, bias, pos0, n, cp, ring, sum);
    if (POOL) {
        // the 4 row groups of a column, added in a fixed order
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float v = sum[h];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) pool_out[(2 * cp + h) * 16 + lane] = v;
        }
    }
}

__global__ __launch_bounds__(kFuseThreads) __attribute__((amdgpu_waves_per_eu(kFuseOcc)))
void nn_fwd_fused_kernel(const uint16_t *X, NnWeights w, const float *P, int32_t n,
                         int32_t tiles, float *zpart)
{
    __shared__ __attribute__((aligned(16))) uint16_t ha[kFuseRows * kFuseStrideH];
    __shared__ __attribute__((aligned(16))) uint16_t hb[kFuseRows * kFuseStrideH];
    uint16_t *xs = hb;  // the input tile, until layer 2 writes hb
    const int tid = threadIdx.x;
    const int t = blockIdx.x / tiles, k = blockIdx.x - t * tiles;
    const int j0 = k * kFuseTP;
    const int cp = tid >> 6;
    constexpr int KB1 = kFuseK1 / 32, KBH = kNnTaps * kNnWidth / 32;
    constexpr int D = kFuseDepth;
    FuseRing ring;
#pragma unroll
    for (int d = 0; d < D; ++d) fuse_frag<kFuseK1>(w.g[0], cp, d, ring.b0[d], ring.b1[d]);
    // input rows: position j0 - 8 + r (zero outside the tour), its 8 features from the packed
    // [T][n][8] input (16 bytes)
    for (int r = tid; r < kFuseRows; r += kFuseThreads) {
        const int pos = j0 - 8 + r;
        u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        if (pos >= 0 && pos < n)
            v = *reinterpret_cast<const u16x8 *>(X + ((long long)t * n + pos) * kNnFeatures);
        *reinterpret_cast<u16x8 *>(xs + r * kFuseStrideX) = v;
    }
    fused_layer<kNnCi0, kFuseMT, 0, kNnWidth, false>(xs, ha, w.g[0], w.g[1], P + nn_off_b(0),
                                                      j0 - 6, n, nullptr, ring);
    fused_layer<kNnWidth, kFuseMT, KB1 % D, kNnWidth, false>(ha, hb, w.g[1], w.g[2],
                                                             P + nn_off_b(1), j0 - 4, n, nullptr,
                                                             ring);
    fused_layer<kNnWidth, kFuseMT, (KB1 + KBH) % D, kNnWidth, false>(
        hb, ha, w.g[2], w.g[3], P + nn_off_b(2), j0 - 2, n, nullptr, ring);
    fused_layer<kNnWidth, kFuseTP / 16, (KB1 + 2 * KBH) % D, 0, true>(
        ha, nullptr, w.g[3], nullptr, P + nn_off_b(3), j0, n,
        zpart + ((long long)t * tiles + k) * kNnWidth, ring);
}

// Head from the per-tile sums: z[c] = (sum over tiles, in order) / n, then as nn_head_fwd_kernel.
__global__ __launch_bounds__(128) void nn_head_pool_kernel(const float *zpart, int32_t tiles,
                                                           int32_t n, const float *P, float *z,
                                                           float *a, float *y, float *pred,
                                                           double shift, double scale)
{
    __shared__ float zs[kNnWidth];
    __shared__ float red[kNnWidth];
    const int t = blockIdx.x, c = threadIdx.x;
    float sum = 0.f;
    for (int k = 0; k < tiles; ++k) sum += zpart[((long long)t * tiles + k) * kNnWidth + c];
    const float zc = sum / (float)n;
    zs[c] = zc;
    z[(long long)t * kNnWidth + c] = zc;
    __syncthreads();
    const float *Wa = P + kNnOffWa;
    float acc = P[kNnOffBa + c];
    for (int i = 0; i < kNnWidth; ++i) acc += Wa[c * kNnWidth + i] * zs[i];
    a[(long long)t * kNnWidth + c] = acc;
    red[c] = P[kNnOffWb + c] * (acc > 0.f ? acc : 0.f);
    __syncthreads();
    for (int off = 64; off > 0; off >>= 1) {
        if (c < off) red[c] += red[c + off];
        __syncthreads();
    }
    if (c == 0) {
        const float yt = red[0] + P[kNnOffBb];
        y[t] = yt;
        if (pred) pred[t] = (float)((double)yt * scale + shift);
    }
}

// ------------------------------------------------------------------------- pool and head

// One workgroup of 256 threads per tour: z = mean over positions of H4, a = Wa z + ba,
// u = relu(a), y = wb . u + bb, pred = y * scale + shift. Thread (r, g) = (tid / 16, tid % 16)
// sums channels 8g .. 8g+7 over positions r, r + 16, ... with 16-byte loads; the 16 partial
// sums of a channel are then added in order r = 0..15 (a fixed order: bitwise reproducible).
__global__ __launch_bounds__(256) void nn_head_fwd_kernel(const uint16_t *H4, int32_t T,
                                                          int32_t n, const float *P, float *z,
                                                          float *a, float *y, float *pred,
                                                          double shift, double scale)
{
    __shared__ float part[16][kNnWidth];
    __shared__ float zs[kNnWidth];
    __shared__ float red[kNnWidth];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int r = tid >> 4, g = tid & 15;
    const u16x8 *h = reinterpret_cast<const u16x8 *>(H4 + ((long long)t * (n + 4) + 2) * kNnWidth) + g;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int j = r;
    for (; j + 48 < n; j += 64) {  // rows j, j + 16, j + 32, j + 48: loads first, adds in order
        u16x8 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = h[(long long)(j + 16 * u) * (kNnWidth / 8)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += bf16_to_f32(v[u][e]);
    }
    for (; j < n; j += 16) {
        const u16x8 v = h[(long long)j * (kNnWidth / 8)];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += bf16_to_f32(v[e]);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) part[r][8 * g + e] = s[e];
    __syncthreads();
    const int c = tid;
    if (c < kNnWidth) {
        float sum = 0.f;
        for (int k = 0; k < 16; ++k) sum += part[k][c];
        const float zc = sum / (float)n;
        zs[c] = zc;
        z[(long long)t * kNnWidth + c] = zc;
    }
    __syncthreads();
    if (c < kNnWidth) {
        const float *Wa = P + kNnOffWa;
        float acc = P[kNnOffBa + c];
        for (int i = 0; i < kNnWidth; ++i) acc += Wa[c * kNnWidth + i] * zs[i];
        a[(long long)t * kNnWidth + c] = acc;
        red[c] = P[kNnOffWb + c] * (acc > 0.f ? acc : 0.f);
    }
    __syncthreads();
    for (int off = 64; off > 0; off >>= 1) {
        if (c < off) red[c] += red[c + off];
        __syncthreads();
    }
    if (c == 0) {
        const float yt = red[0] + P[kNnOffBb];
        y[t] = yt;
        if (pred) pred[t] = (float)((double)yt * scale + shift);
    }
}

// Loss and head backward of a batch: dy_t = 2 (y_t - yhat_t) / T with yhat = (label - shift) /
// scale; da = dy wb [a > 0]; dz = Wa^T da. One workgroup per tour; loss terms per tour.
__global__ __launch_bounds__(128) void nn_head_bwd_kernel(const float *labels, int32_t T,
                                                          const float *P, const float *a,
                                                          const float *y, double shift,
                                                          double scale, float *da, float *dz,
                                                          float *dy, float *loss_terms)
{
    __shared__ float das[kNnWidth];
    const int t = blockIdx.x, c = threadIdx.x;
    const float yhat = (float)(((double)labels[t] - shift) / scale);
    const float err = y[t] - yhat;
    const float d = 2.f * err / (float)T;
    const float at = a[(long long)t * kNnWidth + c];
    const float dac = at > 0.f ? d * P[kNnOffWb + c] : 0.f;
    das[c] = dac;
    da[(long long)t * kNnWidth + c] = dac;
    if (c == 0) {
        dy[t] = d;
        loss_terms[t] = err * err;
    }
    __syncthreads();
    const float *Wa = P + kNnOffWa;
    float s = 0.f;
    for (int o = 0; o < kNnWidth; ++o) s += Wa[o * kNnWidth + c] * das[o];
    dz[(long long)t * kNnWidth + c] = s;
}

// Head parameter gradients, summed over the batch in tour order. Grid kNnWidth + 1 workgroups of
// 128: workgroup o < 128 writes gWa[o][*] and gba[o]; the last writes gwb and gbb.
// The sums run in tour order; the loads of 8 tours are issued before their products.
__global__ __launch_bounds__(128) void nn_head_grad_kernel(int32_t T, const float *__restrict__ z,
                                                           const float *__restrict__ a,
                                                           const float *__restrict__ da,
                                                           const float *__restrict__ dy,
                                                           float *__restrict__ G)
{
    const int o = blockIdx.x, i = threadIdx.x;
    if (o < kNnWidth) {
        float s = 0.f, sb = 0.f;
        int t = 0;
        for (; t + 8 <= T; t += 8) {
            float d[8], zz[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                d[u] = da[(long long)(t + u) * kNnWidth + o];
                zz[u] = z[(long long)(t + u) * kNnWidth + i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s += d[u] * zz[u];
                sb += d[u];
            }
        }
        for (; t < T; ++t) {
            const float d = da[(long long)t * kNnWidth + o];
            s += d * z[(long long)t * kNnWidth + i];
            sb += d;
        }
        G[kNnOffWa + o * kNnWidth + i] = s;
        if (i == 0) G[kNnOffBa + o] = sb;
    } else {
        float s = 0.f, sb = 0.f;
        int t = 0;
        for (; t + 8 <= T; t += 8) {
            float at[8], dd[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                at[u] = a[(long long)(t + u) * kNnWidth + i];
                dd[u] = dy[t + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s += dd[u] * (at[u] > 0.f ? at[u] : 0.f);
                sb += dd[u];
            }
        }
        for (; t < T; ++t) {
            const float at = a[(long long)t * kNnWidth + i];
            s += dy[t] * (at > 0.f ? at : 0.f);
            sb += dy[t];
        }
        G[kNnOffWb + i] = s;
        if (i == 0) G[kNnOffBb] = sb;
    }
}

// dP4[t][j][c] = bf16(dz[t][c] / n) where H4 > 0, else 0 (interior rows only); a thread takes
// 8 consecutive channels of one position (16-byte loads and stores)
__global__ __launch_bounds__(256) void nn_dp4_kernel(const float *__restrict__ dz,
                                                     const uint16_t *__restrict__ H4, int32_t T,
                                                     int32_t n, uint16_t *__restrict__ dP)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;  // (position, channel octet)
    if (e >= (long long)T * n * (kNnWidth / 8)) return;
    const int c0 = (int)(e % (kNnWidth / 8)) * 8;
    const long long m = e / (kNnWidth / 8);
    const long long t = m / n, j = m - t * n;
    const long long idx = (t * (n + 4) + j + 2) * kNnWidth + c0;
    const u16x8 h = *reinterpret_cast<const u16x8 *>(H4 + idx);
    const float *dzt = dz + t * kNnWidth + c0;
    u16x8 out;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool on = h[k] != 0 && !(h[k] & 0x8000u);
        out[k] = on ? bf16_bits_f32(dzt[k] / (float)n) : (uint16_t)0;
    }
    *reinterpret_cast<u16x8 *>(dP + idx) = out;
}

// ------------------------------------------------------------------------- weight gradients

// Partial weight and bias gradients on the matrix cores. The sums run over the padded rows r of
// the batch (R = T (n + 4) rows; the pre-activation gradient dP is zero on every padding row, so
// those rows add nothing): dW[tap][ci][co] = sum_r H[r - 2 + tap][ci] * dP[r][co] and
// db[co] = sum_r dP[r][co]. Workgroup (chunk c, slice s) takes rows 2 + c * chunk .. up to
// R - 2 and input channels 32 s .. 32 s + 31, for every tap and output channel. It stages 64 rows
// at a time in LDS, transposed so that the contracted index (rows) is contiguous: dP^T [co][k],
// and one copy of H^T [ci][k] per tap, shifted by the tap, so that every fragment read is an
// aligned 16-byte load. The workgroup's output channels are those of part h = blockIdx.z of
// 128 / (64 NJ); wave w accumulates NJ 16-channel tiles of them (w NJ 16 ..), for both ci tiles
// and all taps. Slice 0 also sums the bias gradient, one thread per channel over the staged rows
// in order. A channel's sums run in the same order for either NJ (layer 1 takes NJ = 1: its
// single channel slice would otherwise leave half of the compute units idle).
template <int CI, int NJ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void nn_wgrad_kernel(
    const uint16_t *__restrict__ H, const uint16_t *__restrict__ dP, long long R, int32_t chunk,
    float *__restrict__ partW, float *__restrict__ partB)
{
    constexpr int KR = 64;      // rows per staged block
    constexpr int SK = KR + 8;  // bf16 per transposed LDS row (16 bytes of padding)
    constexpr int CW = 64 * NJ;                     // output channels of the workgroup
    constexpr int NP = KR * (CW / 8) / 256;         // dP chunks per thread and block
    constexpr int NH = ((KR + 4) * 4 + 255) / 256;  // H chunks per thread and block (at most)
    static_assert(NJ == 1 || NJ == 2, "one or two output tiles per wavefront");
    __shared__ __attribute__((aligned(16))) uint16_t pt[CW * SK];
    __shared__ __attribute__((aligned(16))) uint16_t ht[kNnTaps * 32 * SK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int slice = blockIdx.y;
    const int co0 = blockIdx.z * CW;  // first output channel of the workgroup
    const long long r0 = 2 + (long long)blockIdx.x * chunk;
    const long long r1 = r0 + chunk < R - 2 ? r0 + chunk : R - 2;
    f32x4 acc[kNnTaps][2][NJ];
#pragma unroll
    for (int t = 0; t < kNnTaps; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[t][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    // a block's global rows, loaded one block ahead: dP rows rb .. rb + 63 (zero from r1 on),
    // CW / 8 chunks of 8 channels per row, and H rows rb - 2 .. rb + 65 (rb >= 2; zero past the
    // last row), 4 chunks of 8 channels of this slice
    u16x8 dv[NP], hv[NH];
    auto load_block = [&](long long rb) {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int e = tid + 256 * u;
            const long long r = rb + e % KR;
            dv[u] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (r < r1)
                dv[u] = *reinterpret_cast<const u16x8 *>(dP + r * kNnWidth + co0 +
                                                          (e / KR) * 8);
        }
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int e = tid + 256 * u;
            const long long h = rb - 2 + e % (KR + 4);
            hv[u] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (e < (KR + 4) * 4 && h < R)
                hv[u] = *reinterpret_cast<const u16x8 *>(H + h * CI + slice * 32 +
                                                          (e / (KR + 4)) * 8);
        }
    };
    if (r0 < r1) load_block(r0);
    for (long long rb = r0; rb < r1; rb += KR) {
        __syncthreads();  // the previous block's fragments have been read
        // dP^T: row k of the block to column k of channel rows c * 8 .. c * 8 + 7
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int e = tid + 256 * u;
            const int k = e % KR, c = e / KR;
#pragma unroll
            for (int i = 0; i < 8; ++i) pt[(c * 8 + i) * SK + k] = dv[u][i];
        }
        // H^T: row rb - 2 + k goes to position k - tap of tap's copy
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int e = tid + 256 * u;
            if (e < (KR + 4) * 4) {
                const int k = e % (KR + 4), c = e / (KR + 4);
#pragma unroll
                for (int t = 0; t < kNnTaps; ++t) {
                    const int kk = k - t;
                    if (kk >= 0 && kk < KR) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) ht[(t * 32 + c * 8 + i) * SK + kk] = hv[u][i];
                    }
                }
            }
        }
        // the next block's rows are in flight while this one is multiplied
        if (rb + KR < r1) load_block(rb + KR);
        __syncthreads();
        if (slice == 0 && tid < CW) {
#pragma unroll
            for (int k = 0; k < KR; k += 8) {
                const u16x8 v = *reinterpret_cast<const u16x8 *>(pt + tid * SK + k);
#pragma unroll
                for (int i = 0; i < 8; ++i) bsum += bf16_to_f32(v[i]);
            }
        }
#pragma unroll
        for (int kb = 0; kb < KR / 32; ++kb) {
            const int kk = kb * 32 + kq * 8;
            bf16x8 b[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                b[j] = *reinterpret_cast<const bf16x8 *>(pt + ((NJ * wave + j) * 16 + r16) * SK +
                                                         kk);
#pragma unroll
            for (int t = 0; t < kNnTaps; ++t) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const bf16x8 a =
                        *reinterpret_cast<const bf16x8 *>(ht + (t * 32 + i * 16 + r16) * SK + kk);
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[t][i][j] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[t][i][j], 0, 0, 0);
                }
            }
        }
    }
    // lane (r16, kq) holds rows ci = 16 i + 4 kq + q, column co = co0 + 16 (NJ wave + j) + r16
    float *dst = partW + (long long)blockIdx.x * (kNnTaps * CI * kNnWidth);
#pragma unroll
    for (int t = 0; t < kNnTaps; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ci = slice * 32 + i * 16 + kq * 4 + q;
                    const int co = co0 + (NJ * wave + j) * 16 + r16;
                    dst[((long long)t * CI + ci) * kNnWidth + co] = acc[t][i][j][q];
                }
    if (slice == 0 && tid < CW) partB[(long long)blockIdx.x * kNnWidth + co0 + tid] = bsum;
}

// sum_{k < chunks} p[k * stride] in chunk order, with the loads of 64 chunks issued before
// their adds (one thread per sum: the time is the latency of these loads). In the last group,
// slots past the last chunk load that chunk again and add +0.0 instead, which leaves every sum
// unchanged (a sum that starts at +0.0 is never -0.0).
__device__ __forceinline__ float sum_chunks(const float *__restrict__ p, long long stride,
                                            int32_t chunks)
{
    float s = 0.f;
    for (int k = 0; k < chunks; k += 64) {
        float v[64];
#pragma unroll
        for (int u = 0; u < 64; ++u) v[u] = p[(long long)min(k + u, chunks - 1) * stride];
#pragma unroll
        for (int u = 0; u < 64; ++u) s += k + u < chunks ? v[u] : 0.f;
    }
    return s;
}

// G[offW + e] = sum over chunks of partW[chunk][e] (e < count), G[offB + c] likewise for the bias
__global__ __launch_bounds__(256) void nn_wgrad_reduce_kernel(const float *__restrict__ partW,
                                                              const float *__restrict__ partB,
                                                              int32_t chunks, int32_t count,
                                                              float *__restrict__ G, int32_t offW,
                                                              int32_t offB)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < count) {
        G[offW + e] = sum_chunks(partW + e, count, chunks);
    } else if (e < count + kNnWidth) {
        const int c = e - count;
        G[offB + c] = sum_chunks(partB + c, kNnWidth, chunks);
    }
}

// ------------------------------------------------------------------------- Adam and weights

__global__ __launch_bounds__(256) void nn_adam_kernel(float *P, float *m, float *v, const float *G,
                                                      int32_t count, float lr, float bc1,
                                                      float bc2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    const float g = G[e];
    const float mm = 0.9f * m[e] + 0.1f * g;
    const float vv = 0.999f * v[e] + 0.001f * g * g;
    m[e] = mm;
    v[e] = vv;
    P[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

// bf16 copies of the conv weights: Wf_l[co][tap * CI + ci] (forward) and, for layers 2..4,
// Wb_l[ci][tap' * 128 + co] = W_l[4 - tap'][ci][co] (backward data). One thread per weight.
// Position of weight (co, k) of a layer with K = 32 KB in MFMA fragment order: the 16-byte
// B operand of lane kq * 16 + r16 for channel tile 2 cp + h and K block kb holds
// k = 32 kb + 8 kq .. + 7 of channel co = (2 cp + h) * 16 + r16; the two tiles of a channel pair
// and the 64 lanes are adjacent, so a wave reads one pair's fragment as 2 x 1 KB contiguous.
__device__ __forceinline__ int nn_frag_index(int co, int k, int KB)
{
    const int cp = co >> 5, h = (co >> 4) & 1, r16 = co & 15;
    const int kb = k >> 5, kq = (k >> 3) & 3, e = k & 7;
    return (((cp * KB + kb) * 2 + h) * 64 + kq * 16 + r16) * 8 + e;
}

__global__ __launch_bounds__(256) void nn_pack_kernel(const float *P, NnWeights w)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    constexpr int n1 = kNnTaps * kNnCi0 * kNnWidth, nl = kNnTaps * kNnWidth * kNnWidth;
    if (e < n1) {
        const int tap = e / (kNnCi0 * kNnWidth), r = e % (kNnCi0 * kNnWidth);
        const int ci = r / kNnWidth, co = r % kNnWidth;
        const uint16_t b = bf16_bits_f32(P[nn_off_w(0) + e]);
        w.f[0][co * (kNnTaps * kNnCi0) + tap * kNnCi0 + ci] = b;
        if (ci < kNnFeatures)  // the fused kernel's packed K (the rest of w.g[0] stays zero)
            w.g[0][nn_frag_index(co, tap * kNnFeatures + ci, kFuseK1 / 32)] = b;
        return;
    }
    const int e2 = e - n1;
    if (e2 >= 3 * nl) return;
    const int l = 1 + e2 / nl, r0 = e2 % nl;
    const int tap = r0 / (kNnWidth * kNnWidth), r = r0 % (kNnWidth * kNnWidth);
    const int ci = r / kNnWidth, co = r % kNnWidth;
    const uint16_t b = bf16_bits_f32(P[nn_off_w(l) + r0]);
    w.f[l][co * (kNnTaps * kNnWidth) + tap * kNnWidth + ci] = b;
    w.b[l][ci * (kNnTaps * kNnWidth) + (kNnTaps - 1 - tap) * kNnWidth + co] = b;
    w.g[l][nn_frag_index(co, tap * kNnWidth + ci, kNnTaps * kNnWidth / 32)] = b;
}

// ------------------------------------------------------------------------- top-k

__device__ __forceinline__ uint32_t nn_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // increasing with f
}

// Histogram of the 8-bit digit `shift` of the keys whose higher digits equal sel->prefix.
__global__ __launch_bounds__(256) void nn_topk_hist_kernel(const float *s, long long C,
                                                           const NnSelect *sel, int shift,
                                                           unsigned long long *hist)
{
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t prefix = sel->prefix, pmask = sel->mask;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < C;
         i += (long long)gridDim.x * 256) {
        const uint32_t k = nn_key(s[i]);
        if ((k & pmask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// One thread: pick the digit where the running count reaches the remaining rank; clear hist.
__global__ void nn_topk_pick_kernel(NnSelect *sel, int shift, unsigned long long *hist)
{
    unsigned long long below = 0;
    int d = 0;
    for (; d < 256; ++d) {
        if (below + hist[d] >= sel->rank) break;
        below += hist[d];
    }
    if (d > 255) d = 255;  // unreachable when rank <= the candidates left
    sel->rank -= below;
    sel->prefix |= (uint32_t)d << shift;
    sel->mask |= 255u << shift;
    for (int k = 0; k < 256; ++k) hist[k] = 0;
}

// Per block of 256 candidates: how many keys are below the threshold and how many equal it.
__global__ __launch_bounds__(256) void nn_topk_count_kernel(const float *s, long long C,
                                                            const NnSelect *sel,
                                                            unsigned int *cnt)
{
    __shared__ unsigned int lt, eq;
    if (threadIdx.x == 0) {
        lt = 0;
        eq = 0;
    }
    __syncthreads();
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < C) {
        const uint32_t k = nn_key(s[i]);
        if (k < sel->prefix) atomicAdd(&lt, 1u);
        else if (k == sel->prefix) atomicAdd(&eq, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt[2 * blockIdx.x] = lt;
        cnt[2 * blockIdx.x + 1] = eq;
    }
}

// One workgroup: exclusive prefix of the per-block counts, in block order. Ties at the threshold
// go to the lowest indices: a block takes min(eq, remaining ties) of them.
__global__ __launch_bounds__(256) void nn_topk_scan_kernel(unsigned int *cnt, long long nblocks,
                                                           const NnSelect *sel,
                                                           unsigned long long *base)
{
    if (threadIdx.x != 0) return;
    unsigned long long pos = 0, ties = sel->rank;  // equal keys still to take
    for (long long b = 0; b < nblocks; ++b) {
        const unsigned long long lt = cnt[2 * b], eq = cnt[2 * b + 1];
        const unsigned long long take_eq = eq < ties ? eq : ties;
        ties -= take_eq;
        base[2 * b] = pos;
        base[2 * b + 1] = take_eq;
        pos += lt + take_eq;
    }
}

// Write the selected indices in increasing index order.
__global__ __launch_bounds__(256) void nn_topk_write_kernel(const float *s, long long C,
                                                            const NnSelect *sel,
                                                            const unsigned long long *base,
                                                            int32_t *idx)
{
    __shared__ unsigned int flags[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    uint32_t f = 0;
    if (i < C) {
        const uint32_t k = nn_key(s[i]);
        f = k < sel->prefix ? 1u : (k == sel->prefix ? 2u : 0u);
    }
    flags[threadIdx.x] = f;
    __syncthreads();
    if (f == 0) return;
    // rank among this block's selected entries (below first, ties by index within the quota)
    unsigned int before = 0, eq_before = 0;
    for (int u = 0; u < (int)threadIdx.x; ++u) {
        if (flags[u] == 2u) ++eq_before;
    }
    const unsigned long long quota = base[2 * blockIdx.x + 1];
    if (f == 2u && eq_before >= quota) return;
    for (int u = 0; u < (int)threadIdx.x; ++u) {
        if (flags[u] == 1u) ++before;
        else if (flags[u] == 2u) before += 1;
    }
    // equal keys beyond the quota that precede this entry are not taken
    const unsigned int skipped = eq_before > quota ? (unsigned int)(eq_before - quota) : 0u;
    idx[base[2 * blockIdx.x] + before - skipped] = (int32_t)i;
}

// ------------------------------------------------------------------------- batches and loss

// dst[b][*] = src[idx[b]][*] (tours of length n) and dlab[b] = lab[idx[b]] when lab is set
__global__ __launch_bounds__(256) void nn_gather_kernel(const int32_t *src, const float *lab,
                                                        const int32_t *idx, int32_t B, int32_t n,
                                                        int32_t *dst, float *dlab)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)B * n) return;
    const long long b = e / n, j = e - b * n;
    const long long r = idx[b];
    dst[e] = src[r * n + j];
    if (lab && j == 0) dlab[b] = lab[r];
}

// *err = 1 if some id of count values lies outside 1..N
__global__ __launch_bounds__(256) void nn_check_ids_kernel(const int32_t *ids, long long count,
                                                           int32_t N, int32_t *err)
{
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < count;
         e += (long long)gridDim.x * 256) {
        const int32_t c = ids[e];
        if (c < 1 || c > N) atomicOr(err, 1);
    }
}

// Candidate tours from one tour and a list of moves, one workgroup per candidate:
// move (0, i, j) reverses positions min(i,j)..max(i,j); move (1, i, j) moves the customer at
// position i to position j. Each output position gathers its customer from the input tour.
__global__ __launch_bounds__(256) void nn_moves_kernel(const int32_t *cur, const int32_t *moves,
                                                       int32_t n, int32_t *out)
{
    const long long c = blockIdx.x;
    const int type = moves[3 * c], i = moves[3 * c + 1], j = moves[3 * c + 2];
    int32_t *dst = out + c * n;
    for (int p = threadIdx.x; p < n; p += 256) {
        int src = p;
        if (type == 0) {
            const int lo = i < j ? i : j, hi = i < j ? j : i;
            if (p >= lo && p <= hi) src = lo + hi - p;
        } else if (i < j) {
            if (p >= i && p < j) src = p + 1;
            else if (p == j) src = i;
        } else {
            if (p > j && p <= i) src = p - 1;
            else if (p == j) src = i;
        }
        dst[p] = cur[src];
    }
}

// out[0] = (sum of terms[0..T-1], in order) / T
__global__ void nn_loss_kernel(const float *terms, int32_t T, float *out)
{
    float s = 0.f;
    for (int t = 0; t < T; ++t) s += terms[t];
    out[0] = s / (float)T;
}

// ------------------------------------------------------------------------- launchers

hipError_t nn_launch_gather(const int32_t *src, const float *lab, const int32_t *idx, int32_t B,
                            int32_t n, int32_t *dst, float *dlab, hipStream_t st)
{
    hipLaunchKernelGGL(nn_gather_kernel, dim3((unsigned)(((long long)B * n + 255) / 256)),
                       dim3(256), 0, st, src, lab, idx, B, n, dst, dlab);
    return hipGetLastError();
}

hipError_t nn_launch_check_ids(const int32_t *ids, long long count, int32_t N, int32_t *err,
                               hipStream_t st)
{
    const long long g = (count + 255) / 256;
    hipLaunchKernelGGL(nn_check_ids_kernel, dim3((unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096)),
                       dim3(256), 0, st, ids, count, N, err);
    return hipGetLastError();
}

hipError_t nn_launch_moves(const int32_t *cur, const int32_t *moves, int32_t count, int32_t n,
                           int32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(nn_moves_kernel, dim3((unsigned)count), dim3(256), 0, st, cur, moves, n,
                       out);
    return hipGetLastError();
}

hipError_t nn_launch_loss(const float *terms, int32_t T, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(nn_loss_kernel, dim3(1), dim3(1), 0, st, terms, T, out);
    return hipGetLastError();
}

static inline unsigned grid_of(long long work, int per) { return (unsigned)((work + per - 1) / per); }

hipError_t nn_launch_dstats(const int16_t *demand, int64_t ld, int64_t S, int32_t N, double *musd,
                            hipStream_t st)
{
    hipLaunchKernelGGL(nn_dstats_kernel, dim3(N), dim3(256), 0, st, demand, ld, S, musd);
    return hipGetLastError();
}

hipError_t nn_launch_features(const NnInstance &in, const int32_t *tours, int32_t T, int32_t n,
                              const double *musd, int32_t Q, double L, uint16_t *X, bool packed,
                              int32_t *err, hipStream_t st)
{
    hipLaunchKernelGGL(nn_features_kernel, dim3(grid_of((long long)T * n, 256)), dim3(256), 0, st,
                       in, tours, T, n, musd, Q, L, X, (int32_t)packed, err);
    return hipGetLastError();
}

hipError_t nn_launch_conv(int ci, int mode, const uint16_t *X, const uint16_t *Wt,
                          const float *bias, const uint16_t *mask, uint16_t *Y, int32_t T,
                          int32_t n, hipStream_t st)
{
    const dim3 g(grid_of((long long)T * n, 256)), b(256);
    if (ci == kNnCi0 && mode == 0)
        hipLaunchKernelGGL((nn_conv_kernel<kNnCi0, 0>), g, b, 0, st, X, Wt, bias, mask, Y, T, n);
    else if (ci == kNnWidth && mode == 0)
        hipLaunchKernelGGL((nn_conv_kernel<kNnWidth, 0>), g, b, 0, st, X, Wt, bias, mask, Y, T, n);
    else if (ci == kNnWidth && mode == 1)
        hipLaunchKernelGGL((nn_conv_kernel<kNnWidth, 1>), g, b, 0, st, X, Wt, bias, mask, Y, T, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int32_t nn_fused_tiles(int32_t n) { return (n + kFuseTP - 1) / kFuseTP; }

hipError_t nn_launch_fwd_fused(const uint16_t *X, const NnWeights &w, const float *P, int32_t T,
                               int32_t n, float *zpart, hipStream_t st)
{
    const int32_t tiles = nn_fused_tiles(n);
    hipLaunchKernelGGL(nn_fwd_fused_kernel, dim3((unsigned)((long long)T * tiles)),
                       dim3(kFuseThreads), 0, st, X, w, P, n, tiles, zpart);
    return hipGetLastError();
}

hipError_t nn_launch_head_pool(const float *zpart, int32_t T, int32_t n, const float *P, float *z,
                               float *a, float *y, float *pred, double shift, double scale,
                               hipStream_t st)
{
    hipLaunchKernelGGL(nn_head_pool_kernel, dim3(T), dim3(128), 0, st, zpart,
                       nn_fused_tiles(n), n, P, z, a, y, pred, shift, scale);
    return hipGetLastError();
}

hipError_t nn_launch_head_fwd(const uint16_t *H4, int32_t T, int32_t n, const float *P, float *z,
                              float *a, float *y, float *pred, double shift, double scale,
                              hipStream_t st)
{
    hipLaunchKernelGGL(nn_head_fwd_kernel, dim3(T), dim3(256), 0, st, H4, T, n, P, z, a, y, pred,
                       shift, scale);
    return hipGetLastError();
}

hipError_t nn_launch_head_bwd(const float *labels, int32_t T, int32_t n, const float *P,
                              const float *z, const float *a, const float *y, double shift,
                              double scale, float *da, float *dz, float *dy, float *loss_terms,
                              const uint16_t *H4, uint16_t *dP4, float *G, hipStream_t st)
{
    hipLaunchKernelGGL(nn_head_bwd_kernel, dim3(T), dim3(128), 0, st, labels, T, P, a, y, shift,
                       scale, da, dz, dy, loss_terms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nn_head_grad_kernel, dim3(kNnWidth + 1), dim3(128), 0, st, T, z, a, da, dy,
                       G);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nn_dp4_kernel, dim3(grid_of((long long)T * n * (kNnWidth / 8), 256)),
                       dim3(256), 0, st, dz, H4, T, n, dP4);
    return hipGetLastError();
}

int32_t nn_wgrad_chunks(int32_t T, int32_t n, int32_t chunk)
{
    const long long rows = (long long)T * (n + 4) - 4;  // rows 2 .. T (n + 4) - 3
    return (int32_t)((rows + chunk - 1) / chunk);
}

hipError_t nn_launch_wgrad(int ci, const uint16_t *H, const uint16_t *dP, int32_t T, int32_t n,
                           int32_t chunk, int32_t chunks, float *partW, float *partB, float *G,
                           int32_t offW, int32_t offB, hipStream_t st)
{
    if (chunks != nn_wgrad_chunks(T, n, chunk)) return hipErrorInvalidValue;
    const long long R = (long long)T * (n + 4);
    const dim3 b(256);
    if (ci == kNnCi0)
        hipLaunchKernelGGL((nn_wgrad_kernel<kNnCi0, 1>), dim3(chunks, 1, 2), b, 0, st, H, dP, R,
                           chunk, partW, partB);
    else if (ci == kNnWidth)
        hipLaunchKernelGGL((nn_wgrad_kernel<kNnWidth, 2>), dim3(chunks, kNnWidth / 32, 1), b, 0,
                           st, H, dP, R, chunk, partW, partB);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int count = kNnTaps * ci * kNnWidth;
    hipLaunchKernelGGL(nn_wgrad_reduce_kernel, dim3(grid_of(count + kNnWidth, 256)), dim3(256), 0,
                       st, partW, partB, chunks, count, G, offW, offB);
    return hipGetLastError();
}

hipError_t nn_launch_adam(float *P, float *m, float *v, const float *G, float lr, float bc1,
                          float bc2, hipStream_t st)
{
    hipLaunchKernelGGL(nn_adam_kernel, dim3(grid_of(kNnParams, 256)), dim3(256), 0, st, P, m, v, G,
                       (int32_t)kNnParams, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t nn_launch_pack(const float *P, const NnWeights &w, hipStream_t st)
{
    const long long total = (long long)kNnTaps * kNnCi0 * kNnWidth +
                            3LL * kNnTaps * kNnWidth * kNnWidth;
    hipLaunchKernelGGL(nn_pack_kernel, dim3(grid_of(total, 256)), dim3(256), 0, st, P, w);
    return hipGetLastError();
}

hipError_t nn_launch_topk(const float *s, long long C, long long K, NnSelect *sel,
                          unsigned long long *hist, unsigned int *cnt, unsigned long long *base,
                          int32_t *idx, hipStream_t st)
{
    const unsigned hg = (unsigned)(C < 256LL * 1024 ? grid_of(C, 256) : 1024);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(nn_topk_hist_kernel, dim3(hg), dim3(256), 0, st, s, C, sel, shift,
                           hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(nn_topk_pick_kernel, dim3(1), dim3(1), 0, st, sel, shift, hist);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const unsigned nb = grid_of(C, 256);
    hipLaunchKernelGGL(nn_topk_count_kernel, dim3(nb), dim3(256), 0, st, s, C, sel, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nn_topk_scan_kernel, dim3(1), dim3(256), 0, st, cnt, (long long)nb, sel,
                       base);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nn_topk_write_kernel, dim3(nb), dim3(256), 0, st, s, C, sel, base, idx);
    (void)K;
    return hipGetLastError();
}

}  // namespace splitgpu
