// Multi-problem step kernels of fdwave: several independent problems advance one
// step in one launch (step_multi_kernel), or walk a whole sweep in one launch whose
// running blocks own fixed sets of tiles and wait only for the neighbouring tiles
// (step_persistent_kernel).  The per-tile work is step_body in fdw_step_body.h.

#include <algorithm>

#include "fdw_batch.h"
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

// Progress of a persistent sweep, group by group.  A group is a column of K
// consecutive chunks of one tile column (the chunks the per-step launches use, each
// marched with its own queue fill), and done[g] counts the steps group g has finished
// in this launch.  A group starts step st once each group its stencil reaches has
// finished step st - 1: those groups wrote the level it reads, and read the level it
// overwrites.  The neighbours are the groups one over along each axis: the in-plane
// halo reaches one tile column left/right (and, in 3D, above/below), the axis-0 queues
// the groups before and after (a group spans at least r planes, except a column's
// last, which ends at the wall, so a mirrored cell past a wall lies in the group
// itself or in such a neighbour).
//
// Waits are bounded: a group that waits longer than `timeout` wall-clock ticks sets
// err, and every wait gives up once err is set, so the launch ends whatever happens.
struct Progress {
    unsigned* done;
    unsigned* err;
    long long timeout;
};

// The XCD (one of the eight chiplets, each with its own L2) this wave runs on: the
// hardware register XCC_ID (hwreg 20, bits 3:0).
constexpr int kMaxXcd = 8;
__device__ __forceinline__ int xcd_id()
{
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kMaxXcd - 1);
}

// Publishes that group `g` finished step `st` (every thread of the block calls it).
// Each wave waits until its loads have returned and its stores have reached the L2
// (the L1 writes through), then one thread stores the progress word.  A neighbour on
// the same XCD reads through that same L2, so the stores are already where it will
// look; only when a neighbour runs on another XCD (`cross`) does an agent-scope
// release (an L2 write-back) first push them to memory, beyond this XCD's L2.  Such a
// write-back walks the XCD's whole L2; the XCD-ordered ranges of groups leave them to
// the few groups at a range's edges.
__device__ __forceinline__ void publish_step(const Progress& pr, int g, int st, bool cross)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (cross) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(pr.done + g, (unsigned)(st + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Waits until each lane's neighbour nb (>= 0; lanes without one pass -1) has finished
// step st - 1, then acquires their writes with one agent-scope acquire (an L1 and L2
// invalidation: a neighbour on another XCD wrote to memory, and this CU's L1 may hold
// stale copies even of a same-XCD neighbour's lines; dropping only the L1, the
// work-group-scope invalidate, proved not enough on this device).  One acquire serves
// the block, whose waves all run on this CU and read after the barrier.  Block-uniform
// result: false when the launch must end.
__device__ __forceinline__ bool wait_neighbours(const Progress& pr, const unsigned* done0, int nb, int st)
{
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    if (nb >= 0) {
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(done0 + nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)st) {
            if (__hip_atomic_load(pr.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                bad = 1;
                break;
            }
            if (wall_clock64() - t0 > pr.timeout) {
                atomicExch(pr.err, 1u);
                bad = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
    return bad == 0;
}

// The blocks of a persistent launch that take part, and how they split by XCD.  Every
// block counts itself in on arrival (word 4); the last of the G blocks to arrive fixes
// the count at G (word 5), and if that does not happen within `window` ticks (the
// device holds fewer blocks at once than the grid has), the first block to notice
// fixes it at the arrivals so far.  A block whose arrival index is below the fixed
// count is running, so work shared among those blocks cannot wait on a block that
// never starts; later blocks leave.  Each block taking part then takes a rank among
// those on its XCD (words 8-15 count them) and counts itself as ranked (word 6); once
// all are ranked, the per-XCD counts are final and every block reads the same ones.
struct Team {
    int part;              // blocks taking part (0: this block leaves)
    int rank;              // this block's rank among its XCD's blocks
    int below;             // blocks taking part on the XCDs numbered below this one's
    int here;              // blocks taking part on this block's XCD
};

__device__ __forceinline__ void join_persistent(unsigned* bar, long long window, long long timeout, Team& tm)
{
    __shared__ int s_part, s_rank, s_below, s_here;
    if (threadIdx.x == 0) {
        unsigned* arrivals = bar + 4;
        unsigned* fixed = bar + 5;
        unsigned* ranked = bar + 6;
        unsigned* per_xcd = bar + 8;
        const unsigned G = gridDim.x;
        const unsigned me = __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (me + 1u == G) {
            unsigned expect = 0u;
            __hip_atomic_compare_exchange_strong(fixed, &expect, G, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        }
        long long t0 = wall_clock64();
        unsigned part;
        while ((part = __hip_atomic_load(fixed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u) {
            if (wall_clock64() - t0 > window) {
                unsigned expect = 0u;
                const unsigned now = __hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_compare_exchange_strong(fixed, &expect, now, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            }
            __builtin_amdgcn_s_sleep(1);
        }
        s_part = 0;
        if (me < part) {
            const int x = xcd_id();
            s_rank = (int)__hip_atomic_fetch_add(per_xcd + x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // release / acquire: a block that sees every block ranked also sees every
            // per-XCD count those blocks added before (relaxed atomics to two words
            // need not land in the order they were issued)
            __hip_atomic_fetch_add(ranked, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            t0 = wall_clock64();
            bool ok = true;
            while (__hip_atomic_load(ranked, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < part) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    wall_clock64() - t0 > timeout) {
                    atomicExch(bar + 2, 1u);
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (ok) {
                int below = 0;
                for (int y = 0; y < x; ++y)
                    below += (int)__hip_atomic_load(per_xcd + y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_below = below;
                s_here = (int)__hip_atomic_load(per_xcd + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_part = (int)part;
            }
        }
    }
    __syncthreads();
    // the same in every lane: kept in scalar registers, so the loops over steps and
    // groups (and the step arguments they load) stay scalar
    tm.part = __builtin_amdgcn_readfirstlane(s_part);
    tm.rank = __builtin_amdgcn_readfirstlane(s_rank);
    tm.below = __builtin_amdgcn_readfirstlane(s_below);
    tm.here = __builtin_amdgcn_readfirstlane(s_here);
}

// A whole sweep of several problems in one launch.  After the join, the blocks pick
// the group size: the first of the host's candidate sizes (chunks per group cand_k[j],
// group starts group_start[j * (nprob + 1) + p], fewer groups with each j) whose
// groups do not outnumber the blocks taking part, so that each block holds one group
// of every step rather than some holding two.  The groups are split into eight
// consecutive ranges, one per XCD, sized by that XCD's blocks; a block takes the
// groups of its XCD's range at its rank, rank + count, ...  Neighbouring groups then
// mostly share an XCD, so their halos meet in one L2 and publishing a step needs no
// L2 write-back; only groups with a neighbour in another range pay it.  Each group is
// marched chunk by chunk, every chunk with its own queue fill, whose loads are in
// flight together, as in the per-step launches.  There is no grid-wide barrier: a
// group waits for its neighbours' previous step only (Progress), so blocks drift apart
// by up to a step and none idles at the end of a step.  Every block handles its groups
// in (step, group) order, each group always in the same block, and a step's work
// depends on the previous step's only, so the waits cannot form a cycle among running
// blocks; the bounded waits end the launch whatever happens.
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
__global__ __launch_bounds__(TZ*(TY / RY)) void step_persistent_kernel(
    const StepArgs* __restrict__ table, const int32_t* __restrict__ cand_k,
    const int32_t* __restrict__ group_start_all, int ncand, int nprob, int nsteps, unsigned* bar,
    long long timeout, long long window)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, 1> SH;
    __shared__ __attribute__((aligned(16))) T lds[SH::LDS];
    Team tm;
    join_persistent(bar, window, timeout, tm);
    if (tm.part == 0) return;
    int j = 0;
    while (j + 1 < ncand && group_start_all[(size_t)j * (nprob + 1) + nprob] > tm.part) ++j;
    const int32_t* group_start = group_start_all + (size_t)j * (nprob + 1);
    const int K = cand_k[j];
    const int total = group_start[nprob];
    const int lo_g = (int)((long long)total * tm.below / tm.part);
    const int hi_g = (int)((long long)total * (tm.below + tm.here) / tm.part);
    Progress pr;
    pr.done = bar + kProgressWords;
    pr.err = bar + 2;
    pr.timeout = timeout;
    for (int st = 0; st < nsteps; ++st) {
        const StepArgs* t = table + (size_t)st * nprob;
        for (int g = lo_g + tm.rank; g < hi_g; g += tm.here) {
            int lo = 0, hi = nprob;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (group_start[mid] <= g) lo = mid;
                else hi = mid;
            }
            const StepArgs a = t[lo];
            const int gl = g - group_start[lo];
            bool cross = false;
            if (a.active) {
                const int ntz = a.ntz, nty = a.nty;
                const int nch = a.nblk / (ntz * nty);
                const int ngr = (nch + K - 1) / K;
                const int tzb = gl % ntz, rest = gl / ntz, tyb = rest % nty, gi = rest / nty;
                // lane i < 2 NDIM watches neighbour i: -z, +z, -x, +x, -y, +y
                const int tid = threadIdx.x;
                int nb = -1;
                if (tid < 2 * NDIM) {
                    const int ax = tid >> 1, dir = (tid & 1) ? 1 : -1;
                    if (ax == 0 && tzb + dir >= 0 && tzb + dir < ntz) nb = gl + dir;
                    if (ax == 1 && gi + dir >= 0 && gi + dir < ngr) nb = gl + dir * ntz * nty;
                    if (ax == 2 && tyb + dir >= 0 && tyb + dir < nty) nb = gl + dir * ntz;
                }
                const int nbg = nb + group_start[lo];   // the neighbour's index among all groups
                cross = __builtin_amdgcn_readfirstlane(__syncthreads_or(nb >= 0 && (nbg < lo_g || nbg >= hi_g))) != 0;
                if (st > 0 && !wait_neighbours(pr, pr.done + group_start[lo], nb, st)) return;
                const int c1 = min(gi * K + K, nch);
                for (int c = gi * K; c < c1; ++c) {
                    __syncthreads();   // the previous chunk's last LDS reads are done
                    step_body<R, T, AT, NDIM, TZ, TY, RY, VZ, 1>(a, (c * nty + tyb) * ntz + tzb, lds);
                }
            }
            publish_step(pr, g, st, cross);   // also orders this group's LDS reads before the next group's writes
        }
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

// Blocks of the persistent grid: the occupancy calculator's blocks per CU for this
// kernel's registers, LDS and block size (waves per SIMD from the VGPR count within the
// 8 a SIMD holds, blocks from those waves and from the LDS per CU), times the CUs,
// rounded down to a multiple of 8.  The figure sizes the grid and the largest group
// plan (about one group per block and step); the blocks that actually run together
// are counted at run time (join_persistent), and the kernel takes the group plan that
// fits them, so a calculator that counts more blocks than the device holds at once
// costs a short wait, not a deadlock.  (The device attribute of resident blocks per
// multiprocessor reports threads per CU over the largest block, 2048 / 1024 = 2, not a
// limit for smaller blocks.)
constexpr long long kJoinWindowTicks = 20000;   // 200 us of the 100 MHz wall clock
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
static hipError_t launch_persistent_one(const StepArgs* t, const GroupPlans& gp, int nprob, int nsteps,
                                        unsigned* bar, long long timeout, hipStream_t s, int* grid_used)
{
    auto kern = step_persistent_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ>;
    const int threads = TZ * (TY / RY);
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int capacity = std::max(8, (per_cu * cus / 8) * 8);
    if (!t) {   // capacity query
        *grid_used = capacity;
        return hipSuccess;
    }
    const int grid = std::min(capacity, ((gp.groups0 + 7) / 8) * 8);
    *grid_used = grid;
    const long long window = kJoinWindowTicks;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, s, t, gp.cand_k, gp.group_start, gp.ncand, nprob,
                       nsteps, bar, timeout, window);
    return hipGetLastError();
}

template <int R, typename T, typename AT>
static hipError_t launch_persistent_rt(int ndim, int variant, const StepArgs* t, const GroupPlans& gp, int nprob,
                                       int nsteps, unsigned* bar, long long to, hipStream_t s, int* g)
{
    if (ndim == 3) {
        switch (variant) {
        case 1: return launch_persistent_one<R, T, AT, 3, 64, 8, 1, 1>(t, gp, nprob, nsteps, bar, to, s, g);
        case 2: return launch_persistent_one<R, T, AT, 3, 64, 8, 1, 2>(t, gp, nprob, nsteps, bar, to, s, g);
        }
    } else {
        switch (variant) {
        case 1: return launch_persistent_one<R, T, AT, 2, 64, 1, 1, 1>(t, gp, nprob, nsteps, bar, to, s, g);
        case 2: return launch_persistent_one<R, T, AT, 2, 64, 1, 1, 2>(t, gp, nprob, nsteps, bar, to, s, g);
        case 4: return launch_persistent_one<R, T, AT, 2, 128, 1, 1, 2>(t, gp, nprob, nsteps, bar, to, s, g);
        case 5: return launch_persistent_one<R, T, AT, 2, 256, 1, 1, 1>(t, gp, nprob, nsteps, bar, to, s, g);
        }
    }
    return hipErrorInvalidValue;
}

template <int R>
static hipError_t launch_persistent_r(int ndim, int dtype, int acc_dtype, int variant, const StepArgs* t,
                                      const GroupPlans& gp, int nprob, int nsteps, unsigned* bar, long long to,
                                      hipStream_t s, int* g)
{
    if (dtype == 1) return launch_persistent_rt<R, double, double>(ndim, variant, t, gp, nprob, nsteps, bar, to, s, g);
    if (acc_dtype == 1) return launch_persistent_rt<R, float, double>(ndim, variant, t, gp, nprob, nsteps, bar, to, s, g);
    return launch_persistent_rt<R, float, float>(ndim, variant, t, gp, nprob, nsteps, bar, to, s, g);
}

hipError_t launch_step_persistent(int ndim, int r, int dtype, int acc_dtype, int variant, const StepArgs* d_table,
                                  const GroupPlans& gp, int nprob, int nsteps, unsigned* d_progress,
                                  long long timeout_ticks, hipStream_t s, int* grid_used)
{
    switch (r) {
    case 1: return launch_persistent_r<1>(ndim, dtype, acc_dtype, variant, d_table, gp, nprob, nsteps, d_progress, timeout_ticks, s, grid_used);
    case 2: return launch_persistent_r<2>(ndim, dtype, acc_dtype, variant, d_table, gp, nprob, nsteps, d_progress, timeout_ticks, s, grid_used);
    case 4: return launch_persistent_r<4>(ndim, dtype, acc_dtype, variant, d_table, gp, nprob, nsteps, d_progress, timeout_ticks, s, grid_used);
    }
    return hipErrorInvalidValue;
}

hipError_t persistent_capacity(int ndim, int r, int dtype, int acc_dtype, int variant, int* blocks)
{
    const GroupPlans none = {nullptr, nullptr, 0, 0};
    return launch_step_persistent(ndim, r, dtype, acc_dtype, variant, nullptr, none, 0, 0, nullptr, 0, nullptr,
                                  blocks);
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
