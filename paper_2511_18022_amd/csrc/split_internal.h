// Internal interface between the C-ABI host layer (split_host.cpp) and the HIP kernels
// (split_kernels.hip). Not installed; callers use include/split.h.
//
// Every evaluation is a batch of T >= 1 giant tours over one instance and one demand matrix
// (split_eval is the batch of one). Per-tour arrays are concatenated: tour t's positions are
// tours[tptr[t] .. tptr[t+1]) and its derived arrays start at abase(t) = tptr[t] + t * (1 +
// kRowPad), each holding n_t + 1 + kRowPad entries.
//
// The kernels read T from device memory (the staged header), and their grids are sized for an
// upper bound of T: one captured HIP graph then serves every batch up to its capacity.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/split.h"

namespace splitgpu {

// Context accessors for the other host modules of the library (defined in split_host.cpp).
int ctx_device(const split_ctx *ctx);
// false when no instance is set
bool ctx_instance(const split_ctx *ctx, int32_t *N, int *kind, const int32_t **xy,
                  const int32_t **dist, int64_t *max_arc);
// records the message as the context's last error and returns st
split_status ctx_fail(split_ctx *ctx, split_status st, const char *fmt, ...);

// "Infinity" for DP values. Host checks guarantee |DP value| + |weight| < 2^30.
constexpr int32_t kInf = 0x3fffffff;

// Cost mark of a scenario the lane kernel leaves to the general kernel (costs are >= 0).
constexpr int32_t kCostOvf = INT32_MIN;

// Device-side result block of one tour (zeroed by the prep kernel of each call).
struct DevStats {
    unsigned long long sum;    // sum of costs
    unsigned long long sq_lo;  // sum of squared costs, low 64 bits
    unsigned long long sq_hi;  // sum of squared costs, high 64 bits
    int32_t err_demand;        // nonzero: some scenario has q > Q (or q < 0) on the tour
    int32_t ovf_count;         // scenarios of this tour finished by the general kernel
};

// Batch-wide counters (reset by the prep kernel of each call).
struct BatchCtl {
    uint32_t head;       // next work item of the lane kernel's queue
    uint32_t ovf_total;  // scenarios marked kCostOvf, over all tours
};

// Per-tour arrays built on the device by the prep kernel from the tours and the instance.
//   w[0]   = c(0, s_1)                                    (g_0 = f_0 + a_0)
//   w[i]   = c(s_i, 0) + c(0, s_{i+1}) - c(s_i, s_{i+1})   1 <= i <= n-1
//   w[n]   = D[n] + c(s_n, 0)                             (turns g back into f at i = n)
//   rowoff[i] = (s_i - 1) * ld * 2   (byte offset of position i's int16 demand row), 1 <= i <= n
// With g_p = f_p + c(0, s_{p+1}) - D[p+1] (D[k] = tour arc sum up to position k), Eq. (3)
// becomes g_i = w_i + min_{p in window(i)} g_p, and f_n = w_n + min_{p in window(n)} g_p.
// Each array carries kRowPad entries past position n (rowoff: a valid row; rowoff32: absent;
// w: zero) so that the kernels can read whole blocks of positions, up to six blocks past n,
// without guards.
constexpr int kRowPad = 128;

// rowoff32 value of a position without a demand (position 0, positions past n): beyond every
// lane_bytes, so the lane kernel's range-checked buffer loads return 0 for it.
constexpr uint32_t kRowAbsent = 0xFFFFFF00u;

__host__ __device__ inline int64_t tour_abase(const int64_t *tptr, int t)
{
    return tptr[t] + (int64_t)t * (1 + kRowPad);
}

// Staged header, uploaded before every evaluation: int64 T, int64 tptr[T + 1], int32 order[T]
// (the lane kernel's work order), int32 tours[tptr[T]], each part at an offset fixed by the
// capacity the buffers were laid out for.
struct TourDev {
    const int64_t *nt;     // [1] number of tours T of this evaluation
    const int32_t *tours;  // [tptr[T]] concatenated tours
    const int64_t *tptr;   // [T + 1]
    const int32_t *order;  // [T] work order of the lane kernel
    int32_t T_grid;        // upper bound of T that the launch grids are sized for
    int64_t *rowoff;       // concatenated, see above
    uint32_t *rowoff32;    // rowoff mod 2^32 (exact where it is used), kRowAbsent where absent
    int32_t *w;
};

struct PrepArgs {
    TourDev tour;
    int32_t N;
    int32_t kind;          // 0: coordinates, 1: distance matrix
    const int32_t *xy;     // device [(N+1)*2]
    const int32_t *dist;   // device [(N+1)^2]
    int64_t ld;
    DevStats *stats;       // [T]
    BatchCtl *ctl;
};

struct EvalArgs {
    const uint16_t *demand;  // device, row-major [N][ld], read as unsigned (q > Q rejects q < 0)
    int64_t ld;
    int64_t S;
    int32_t Q;
    TourDev tour;
    int32_t *cost;           // device [T][ldc]
    int64_t ldc;
    DevStats *stats;         // [T]
    BatchCtl *ctl;
    uint32_t lane_bytes;     // lane kernel: bytes of demand it may address, <= kRowAbsent
    int32_t lane_grid;       // lane kernel workgroups (>= the work items: one item each)
    int32_t lane_static;     // lane kernel, fewer workgroups than items: 1 = each takes items
                             // at a fixed stride of lane_grid, 0 = from the queue
    int32_t lane_uniform;    // lane kernel: 1 = every tour of the launch has the same length
    int32_t lane_block;      // lane kernel block length: 16 or 8 states
    int32_t wave_grid;       // wave kernel workgroups of a full evaluation (form wave)
    int32_t maxn;            // bound on the tour lengths (sizes the wave kernel's LDS)
};

struct MomentArgs {
    const int32_t *cost;           // [T][ldc]
    int64_t ldc;
    int64_t S;
    const int64_t *nt;             // [1] T
    int32_t T_grid;
    unsigned long long *partials;  // [T][nblocks][3]
    int32_t nblocks;               // per tour
    DevStats *stats;               // [T]
};

// Kernel launchers (split_kernels.hip). All are asynchronous on `stream`.
hipError_t launch_prep(const PrepArgs &a, hipStream_t stream);
hipError_t launch_lane(const EvalArgs &a, hipStream_t stream);
hipError_t launch_wave_all(const EvalArgs &a, hipStream_t stream);
hipError_t launch_wave_fallback(const EvalArgs &a, hipStream_t stream);
hipError_t launch_moments(const MomentArgs &a, hipStream_t stream);
// two-kernel form: mask int16 [rows][mask_ld], row abase(t) + i
hipError_t launch_mask(const EvalArgs &a, int16_t *mask, long long mask_ld, hipStream_t stream);
hipError_t launch_masked_dp(const EvalArgs &a, const int16_t *mask, long long mask_ld,
                            hipStream_t stream);
const char *mask_kernel_name();
int32_t moment_blocks(int64_t S);
const char *lane_kernel_name();
const char *wave_kernel_name();

// Device scratch of the allocation-free evaluation: kScratchBytes per GPU, 256-byte aligned.
// scratch_address returns its device address on `device`, which must be the current device
// (looked up once per device, then cached).
constexpr size_t kScratchBytes = 192 * 1024;
constexpr int kMaxScratchDevices = 64;
hipError_t scratch_address(int device, void **out);

}  // namespace splitgpu
