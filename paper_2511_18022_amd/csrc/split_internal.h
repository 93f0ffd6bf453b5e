// Internal interface between the C-ABI host layer (split_host.cpp) and the HIP kernels
// (split_kernels.hip). Not installed; callers use include/split.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace splitgpu {

// "Infinity" for DP values. Host checks guarantee |DP value| + |weight| < 2^30.
constexpr int32_t kInf = 0x3fffffff;

// Device-side result block of one evaluation (zeroed by the prep kernel of each call).
struct DevStats {
    unsigned long long sum;    // sum of costs
    unsigned long long sq_lo;  // sum of squared costs, low 64 bits
    unsigned long long sq_hi;  // sum of squared costs, high 64 bits
    int32_t err_demand;        // nonzero: some scenario has q > Q (or q < 0) on the tour
    int32_t ovf_count;         // scenarios queued for the general kernel
};

// Per-tour arrays built on the device by the prep kernel from the tour and the instance.
//   w[0]   = c(0, s_1)                                    (g_0 = f_0 + a_0)
//   w[i]   = c(s_i, 0) + c(0, s_{i+1}) - c(s_i, s_{i+1})   1 <= i <= n-1
//   w[n]   = D[n] + c(s_n, 0)                             (turns g back into f at i = n)
//   rowoff[i] = (s_i - 1) * ld * 2   (byte offset of position i's int16 demand row), 1 <= i <= n
// With g_p = f_p + c(0, s_{p+1}) - D[p+1] (D[k] = tour arc sum up to position k), Eq. (3)
// becomes g_i = w_i + min_{p in window(i)} g_p, and f_n = w_n + min_{p in window(n)} g_p.
// Both arrays carry kRowPad entries past position n (rowoff: a valid row; w: zero) so that the
// kernels can read whole blocks of positions, up to six blocks past n, without guards.
constexpr int kRowPad = 128;

struct TourDev {
    int64_t *rowoff;     // [n + 1 + kRowPad]
    uint32_t *rowoff32;  // [n + 1 + kRowPad], rowoff mod 2^32 (exact when it is used);
                         // kRowAbsent at position 0 and past n
    int32_t *w;          // [n + 1 + kRowPad]
};

struct PrepArgs {
    const int32_t *tour;  // device [n]
    int32_t n;
    int32_t N;
    int32_t kind;         // 0: coordinates, 1: distance matrix
    const int32_t *xy;    // device [(N+1)*2]
    const int32_t *dist;  // device [(N+1)^2]
    int64_t ld;
    TourDev out;
    DevStats *stats;
};

struct EvalArgs {
    const uint16_t *demand;  // device, row-major [N][ld], read as unsigned (q > Q rejects q < 0)
    int64_t ld;
    int64_t S;
    int32_t n;
    int32_t Q;
    TourDev tour;
    int32_t *cost;           // device [S]
    DevStats *stats;
    int32_t *ovf_list;       // device [S]: scenarios handed to the general kernel
    uint32_t lane_bytes;     // lane kernel: bytes of demand it may address, <= kRowAbsent
};

// rowoff32 value of a position without a demand (position 0, positions past n): beyond every
// lane_bytes, so the lane kernel's range-checked buffer loads return 0 for it.
constexpr uint32_t kRowAbsent = 0xFFFFFF00u;

struct MomentArgs {
    const int32_t *cost;
    int64_t S;
    unsigned long long *partials;  // [3 * nblocks]
    int32_t nblocks;
    DevStats *stats;
};

// Kernel launchers (split_kernels.hip). All are asynchronous on `stream`.
hipError_t launch_prep(const PrepArgs &a, hipStream_t stream);
hipError_t launch_lane(const EvalArgs &a, hipStream_t stream);
hipError_t launch_wave_all(const EvalArgs &a, hipStream_t stream);
hipError_t launch_wave_fallback(const EvalArgs &a, hipStream_t stream);
hipError_t launch_moments(const MomentArgs &a, hipStream_t stream);
int32_t moment_blocks(int64_t S);
const char *lane_kernel_name();
const char *wave_kernel_name();

}  // namespace splitgpu
