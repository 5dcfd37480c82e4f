// Multi-problem step kernels of fdwave: several independent problems advance one
// step in one launch (step_multi_kernel), or walk a whole sweep in one cooperative
// launch with a bounded grid barrier between steps (step_persistent_kernel).  The
// per-tile work is step_body in fdw_step_body.h.

#include <algorithm>

#include "fdw_step_body.h"

namespace fdw {

// Several problems in one launch: the logical block picks its problem from the
// prefix table block_start (binary search), then runs that problem's tile.
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
__global__ __launch_bounds__(TZ*(TY / RY)) void step_multi_kernel(const StepArgs* __restrict__ table,
                                                                  const int32_t* __restrict__ block_start,
                                                                  int nprob, int total)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, 1> SH;
    __shared__ __attribute__((aligned(16))) T lds[SH::LDS];
    const int g = logical_block(total);
    if (g >= total) return;
    int lo = 0, hi = nprob;   // largest p with block_start[p] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (block_start[mid] <= g) lo = mid;
        else hi = mid;
    }
    const StepArgs a = table[lo];
    if (!a.active) return;
    step_body<R, T, AT, NDIM, TZ, TY, RY, VZ, 1>(a, g - block_start[lo], lds);
}

// Grid-wide barrier with a bounded wait.  bar[0] counts arrivals, bar[1] is the
// generation, bar[2] an error flag.  A block that waits longer than `timeout`
// wall-clock ticks sets the flag and gives up; every block checks the flag after
// each barrier and leaves, so the launch always ends even if some blocks could not
// be resident at once.  Returns false when the caller must leave.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, long long timeout)
{
    __shared__ int leave;
    __syncthreads();
    if (threadIdx.x == 0) {
        int err = 0;
        const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = atomicAdd(bar, 1u) + 1u;
        if (arrived == nblocks) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const long long t0 = wall_clock64();
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                if (wall_clock64() - t0 > timeout) {
                    atomicExch(bar + 2, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        err = __hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        leave = err;
    }
    __syncthreads();
    return !leave;
}

// A whole sweep of several problems in one launch: the resident blocks walk the
// sweep's steps; within a step each block takes the logical blocks slot, slot + G,
// ... (slot remapped so consecutive tiles share an XCD), and a bounded grid barrier
// separates the steps.  Launched cooperatively with a grid sized well inside the
// resident capacity; the bounded barrier is the exit condition if residency fails.
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
__global__ __launch_bounds__(TZ*(TY / RY)) void step_persistent_kernel(
    const StepArgs* __restrict__ table, const int32_t* __restrict__ block_start, int nprob,
    int total, int nsteps, unsigned* bar, long long timeout)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, 1> SH;
    __shared__ __attribute__((aligned(16))) T lds[SH::LDS];
    const int G = gridDim.x;
    const int slot = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);   // G is a multiple of 8
    for (int st = 0; st < nsteps; ++st) {
        const StepArgs* t = table + (size_t)st * nprob;
        for (int g = slot; g < total; g += G) {
            int lo = 0, hi = nprob;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (block_start[mid] <= g) lo = mid;
                else hi = mid;
            }
            const StepArgs a = t[lo];
            if (!a.active) continue;
            __syncthreads();   // the previous tile's last LDS reads are done
            step_body<R, T, AT, NDIM, TZ, TY, RY, VZ, 1>(a, g - block_start[lo], lds);
        }
        if (!grid_barrier(bar, (unsigned)G, timeout)) return;
    }
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
static hipError_t launch_multi_one(const StepArgs* t, const int32_t* bs, int nprob, int total,
                                   hipStream_t s)
{
    const int grid = ((total + 7) / 8) * 8;
    hipLaunchKernelGGL((step_multi_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ>), dim3(grid),
                       dim3(TZ * (TY / RY)), 0, s, t, bs, nprob, total);
    return hipGetLastError();
}

template <int R, typename T, typename AT>
static hipError_t launch_multi_rt(int ndim, int variant, const StepArgs* t, const int32_t* bs,
                                  int nprob, int total, hipStream_t s)
{
    if (ndim == 3) {
        switch (variant) {
        case 1: return launch_multi_one<R, T, AT, 3, 64, 8, 1, 1>(t, bs, nprob, total, s);
        case 2: return launch_multi_one<R, T, AT, 3, 64, 8, 1, 2>(t, bs, nprob, total, s);
        }
    } else {
        switch (variant) {
        case 1: return launch_multi_one<R, T, AT, 2, 64, 1, 1, 1>(t, bs, nprob, total, s);
        case 2: return launch_multi_one<R, T, AT, 2, 64, 1, 1, 2>(t, bs, nprob, total, s);
        case 4: return launch_multi_one<R, T, AT, 2, 128, 1, 1, 2>(t, bs, nprob, total, s);
        case 5: return launch_multi_one<R, T, AT, 2, 256, 1, 1, 1>(t, bs, nprob, total, s);
        }
    }
    return hipErrorInvalidValue;
}

// Resident blocks per CU of the persistent grid: the smallest of what the occupancy
// calculator allows for the kernel's registers and LDS, the device's limit of resident
// blocks per CU, and kPersistentBlocksPerCU.
constexpr int kPersistentBlocksPerCU = 8;
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
static hipError_t launch_persistent_one(const StepArgs* t, const int32_t* bs, int nprob, int total,
                                        int nsteps, unsigned* bar, long long timeout, hipStream_t s,
                                        int* grid_used)
{
    auto kern = step_persistent_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ>;
    const int threads = TZ * (TY / RY);
    int per_cu = 0, dev = 0, cus = 0, slots = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&slots, hipDeviceAttributeMaxBlocksPerMultiProcessor, dev)) != hipSuccess)
        return e;
    if (slots > 0) per_cu = std::min(per_cu, slots);
    per_cu = std::min(per_cu, kPersistentBlocksPerCU);
    int grid = per_cu * cus;
    grid = std::min(grid, ((total + 7) / 8) * 8);
    grid = (grid / 8) * 8;
    if (grid < 8) return hipErrorInvalidConfiguration;
    *grid_used = grid;
    void* args[] = {(void*)&t, (void*)&bs, (void*)&nprob, (void*)&total, (void*)&nsteps,
                    (void*)&bar, (void*)&timeout};
    return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(threads), args, 0, s);
}

template <int R, typename T, typename AT>
static hipError_t launch_persistent_rt(int ndim, int variant, const StepArgs* t, const int32_t* bs,
                                       int nprob, int total, int nsteps, unsigned* bar, long long to,
                                       hipStream_t s, int* g)
{
    if (ndim == 3) {
        switch (variant) {
        case 1: return launch_persistent_one<R, T, AT, 3, 64, 8, 1, 1>(t, bs, nprob, total, nsteps, bar, to, s, g);
        case 2: return launch_persistent_one<R, T, AT, 3, 64, 8, 1, 2>(t, bs, nprob, total, nsteps, bar, to, s, g);
        }
    } else {
        switch (variant) {
        case 1: return launch_persistent_one<R, T, AT, 2, 64, 1, 1, 1>(t, bs, nprob, total, nsteps, bar, to, s, g);
        case 2: return launch_persistent_one<R, T, AT, 2, 64, 1, 1, 2>(t, bs, nprob, total, nsteps, bar, to, s, g);
        case 4: return launch_persistent_one<R, T, AT, 2, 128, 1, 1, 2>(t, bs, nprob, total, nsteps, bar, to, s, g);
        case 5: return launch_persistent_one<R, T, AT, 2, 256, 1, 1, 1>(t, bs, nprob, total, nsteps, bar, to, s, g);
        }
    }
    return hipErrorInvalidValue;
}

template <int R>
static hipError_t launch_persistent_r(int ndim, int dtype, int acc_dtype, int variant, const StepArgs* t,
                                      const int32_t* bs, int nprob, int total, int nsteps, unsigned* bar,
                                      long long to, hipStream_t s, int* g)
{
    if (dtype == 1) return launch_persistent_rt<R, double, double>(ndim, variant, t, bs, nprob, total, nsteps, bar, to, s, g);
    if (acc_dtype == 1) return launch_persistent_rt<R, float, double>(ndim, variant, t, bs, nprob, total, nsteps, bar, to, s, g);
    return launch_persistent_rt<R, float, float>(ndim, variant, t, bs, nprob, total, nsteps, bar, to, s, g);
}

hipError_t launch_step_persistent(int ndim, int r, int dtype, int acc_dtype, int variant,
                                  const StepArgs* d_table, const int32_t* d_block_start, int nprob,
                                  int total_blocks, int nsteps, unsigned* d_barrier,
                                  long long timeout_ticks, hipStream_t s, int* grid_used)
{
    switch (r) {
    case 1: return launch_persistent_r<1>(ndim, dtype, acc_dtype, variant, d_table, d_block_start, nprob, total_blocks, nsteps, d_barrier, timeout_ticks, s, grid_used);
    case 2: return launch_persistent_r<2>(ndim, dtype, acc_dtype, variant, d_table, d_block_start, nprob, total_blocks, nsteps, d_barrier, timeout_ticks, s, grid_used);
    case 4: return launch_persistent_r<4>(ndim, dtype, acc_dtype, variant, d_table, d_block_start, nprob, total_blocks, nsteps, d_barrier, timeout_ticks, s, grid_used);
    }
    return hipErrorInvalidValue;
}

template <int R>
static hipError_t launch_multi_r(int ndim, int dtype, int acc_dtype, int variant, const StepArgs* t,
                                 const int32_t* bs, int nprob, int total, hipStream_t s)
{
    if (dtype == 1) return launch_multi_rt<R, double, double>(ndim, variant, t, bs, nprob, total, s);
    if (acc_dtype == 1) return launch_multi_rt<R, float, double>(ndim, variant, t, bs, nprob, total, s);
    return launch_multi_rt<R, float, float>(ndim, variant, t, bs, nprob, total, s);
}

hipError_t launch_step_multi(int ndim, int r, int dtype, int acc_dtype, int variant,
                             const StepArgs* d_table, const int32_t* d_block_start, int nprob,
                             int total_blocks, hipStream_t s)
{
    switch (r) {
    case 1: return launch_multi_r<1>(ndim, dtype, acc_dtype, variant, d_table, d_block_start, nprob, total_blocks, s);
    case 2: return launch_multi_r<2>(ndim, dtype, acc_dtype, variant, d_table, d_block_start, nprob, total_blocks, s);
    case 4: return launch_multi_r<4>(ndim, dtype, acc_dtype, variant, d_table, d_block_start, nprob, total_blocks, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace fdw
