// The fused leapfrog step of fdwave for gfx950 (CDNA4, wave64).
//
// One step of the scheme (paper Sec. 3.1, Eq. FDstencil2 with rho^-1 = 1,
// kappa = c^2, order-2r Laplacian) over the whole grid, fused with the work that
// Alg. 1 does per time step: source injection (line 4), receiver sampling, the
// residual / adjoint force (line 5) and the kernel increments K(u,u) (line 7) or
// K(v,v) (line 14).  One launch per time step; 2D and 3D share the code.
//
// Layout of the work:
//  * a block owns a tile of the planes normal to axis 0 (3D: TY x WZ cells of
//    axes 1 and 2; 2D: WZ cells of axis 1) and marches along axis 0 through a
//    chunk of planes;
//  * a lane owns VZ consecutive cells of the contiguous axis (WZ = 64 VZ per
//    wave row), so every global access of a wave is one coalesced row segment
//    of 256 VZ bytes (f32) issued as dword, dwordx2 or dwordx4 loads;
//  * a lane advances S shots of the same medium at once: c and the shared
//    accumulator are read once per cell for all S wavefields;
//  * each lane keeps the 2r+1 values of its column along axis 0 in registers
//    (a rotating queue), so axis-0 neighbours cost no extra reads;
//  * the current plane is staged in LDS with an r-wide halo for the in-plane
//    neighbours (cross-shaped stencil: no corner halo), double-buffered so one
//    barrier per plane suffices;
//  * software pipelining: every load of plane x+1 (queue entry x+1+r, halo,
//    u^{n-1}, c, accumulator) is issued before plane x is computed, so a whole
//    plane of work covers the memory latency;
//  * plane bases are wave-uniform 64-bit pointers, in-plane offsets 32-bit;
//  * u^{n+1} overwrites u^{n-1} in place and the speed c is read instead of a
//    stored dt^2 c^2 array, so a step streams four arrays; those streams are read
//    and written non-temporally, which leaves the cache to the u^n halos;
//  * block ids are remapped so that consecutive tiles run on the same XCD
//    (dispatch is round-robin over the 8 XCDs) and share halo rows in its L2.
//
// Difference form of the Laplacian, sum_j w_j [(u_{+j} - u_0) + (u_{-j} - u_0)]:
// L applied to a constant is exactly zero in f32 even though the rounded weights
// do not sum to zero, which removes the phase drift of the a_0 form.

#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "fdw_internal.h"

namespace fdw {

// Ghost index: half-sample mirror about the wall faces, then clamped into the
// array (the clamp only matters for tile-overhang lanes, which store nothing).
__device__ __forceinline__ int ghost(int i, int n)
{
    i = i < 0 ? -1 - i : i;
    i = i >= n ? 2 * n - 1 - i : i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <typename T, int V>
struct Vec { typedef T __attribute__((ext_vector_type(V))) type; };
template <typename T>
struct Vec<T, 1> { typedef T type; };

template <typename T, int V>
__device__ __forceinline__ T el(const typename Vec<T, V>::type& v, int i)
{
    if constexpr (V == 1) return v;
    else return v[i];
}
template <typename T, int V>
__device__ __forceinline__ void set_el(typename Vec<T, V>::type& v, int i, T x)
{
    if constexpr (V == 1) v = x;
    else v[i] = x;
}

template <typename T, int V>
__device__ __forceinline__ typename Vec<T, V>::type reversed(const typename Vec<T, V>::type& v)
{
    if constexpr (V == 1) return v;
    else if constexpr (V == 2) return __builtin_shufflevector(v, v, 1, 0);
    else return __builtin_shufflevector(v, v, 3, 2, 1, 0);
}

// V consecutive cells of one row starting at z (z and the row length n2 are multiples
// of V), without a branch around the load.  A lane past the wall (z >= n2) reads the
// aligned vector that holds its mirrored ghost cells and, when MIRROR, reverses it:
// cell z + i maps to 2 n2 - 1 - z - i.  Without MIRROR such lanes get in-bounds values
// they never use.
template <typename T, int V, bool STREAM, bool MIRROR>
__device__ __forceinline__ typename Vec<T, V>::type load_row(const T* row, int z, int n2)
{
    typedef typename Vec<T, V>::type vec;
    const bool past = z >= n2;
    const int zs = max(past ? 2 * n2 - z - V : z, 0);
    vec v;
    if constexpr (STREAM) v = __builtin_nontemporal_load((const vec*)(row + zs));
    else v = *(const vec*)(row + zs);
    if constexpr (MIRROR && V > 1) v = past ? reversed<T, V>(v) : v;
    return v;
}

// Compile-time shape of one kernel variant.
template <int R, typename T, int NDIM, int TZ, int TY, int RY, int VZ, int S>
struct Shape {
    static constexpr int TYT = TY / RY;            // thread rows; a thread owns RY tile rows
    static constexpr int NT = TZ * TYT;            // threads per block
    static constexpr int WZ = TZ * VZ;             // tile width in cells
    static constexpr int RYH = (NDIM == 3) ? R : 0;
    static constexpr int PADL = VZ * ((R + VZ - 1) / VZ);   // left pad keeps rows VZ-aligned
    static constexpr int LZ = PADL + WZ + PADL;
    static constexpr int LSZ = (TY + 2 * RYH) * LZ;          // one plane of one shot
    static constexpr int HYV = (NDIM == 3) ? 2 * R * TZ : 0; // halo row vectors above and below
    static constexpr int HZ = 2 * R * TY;                    // halo cells left and right
    static constexpr int NHY = (HYV + NT - 1) / NT;
    static constexpr int NHZ = (HZ + NT - 1) / NT;
    static constexpr int NHY1 = NHY > 0 ? NHY : 1;
    static constexpr int LDS = 2 * S * LSZ;                  // double buffer, all shots
};

// One block's share of one step: logical block b of problem `a`.
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, int S>
__device__ __forceinline__ void step_body(const StepArgs& a, const int b, T* __restrict__ lds)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, S> SH;
    typedef typename Vec<T, VZ>::type vec;
    typedef typename Vec<AT, VZ>::type avec;
    constexpr int TYT = SH::TYT, NT = SH::NT, WZ = SH::WZ, RYH = SH::RYH, PADL = SH::PADL;
    constexpr int LZ = SH::LZ, LSZ = SH::LSZ, HYV = SH::HYV, HZ = SH::HZ;
    constexpr int NHY = SH::NHY, NHZ = SH::NHZ, NHY1 = SH::NHY1;

    const int tzb = b % a.ntz;
    const int rest = b / a.ntz;
    const int tyb = rest % a.nty;
    const int chb = rest / a.nty;

    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int z0 = tzb * WZ, y0 = tyb * TY;
    const int x0 = chb * a.chunk_len;
    const int x1 = min(x0 + a.chunk_len, n0);
    const int tid = threadIdx.x;
    const int lz = tid % TZ;
    const int lyt = tid / TZ;
    const int z = z0 + lz * VZ;              // first cell of this lane
    const bool zlive = z < n2;
    const int64_t ps = (int64_t)n1 * n2;
    const int64_t sst = a.shot_stride;

    const T* __restrict__ ucur = (const T*)a.ucur;
    T* __restrict__ unew = (T*)a.unew;
    const T* __restrict__ cc = (const T*)a.c;
    AT* __restrict__ acc = (AT*)a.acc;
    const bool use_acc = a.acc_sign != 0;
    T w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) w[j] = (T)a.w[j];
    const T dt2 = (T)a.dt2;

    // own cells: row offset within a plane (ghosted for overhang rows, which never store)
    int roff[RY], lofs[RY], lane0[RY];
    bool live[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        const int ly = lyt + k * TYT;
        const int y = y0 + ly;
        roff[k] = ghost(y, n1) * n2;
        live[k] = zlive && (y < n1);
        lofs[k] = (ly + RYH) * LZ + PADL + lz * VZ;
        lane0[k] = ly * WZ + lz * VZ;
    }
    // halo rows (3D): LDS slot of the vector and its row offset in the plane
    int hyl[NHY1], hyr[NHY1], hyz[NHY1];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int h = tid + i * NT;
        const int row = h / TZ;
        const int sy = row < R ? row : row + TY;
        const int cz = (h % TZ) * VZ;
        hyl[i] = h < HYV ? sy * LZ + PADL + cz : -1;
        hyr[i] = ghost(y0 + sy - R, n1) * n2;
        hyz[i] = z0 + cz;
    }
    // halo columns: LDS slot and in-plane offset of single cells
    int hzl[NHZ], hzg[NHZ];
#pragma unroll
    for (int i = 0; i < NHZ; ++i) {
        const int h = tid + i * NT;
        const int row = h / (2 * R);
        const int col = h % (2 * R);
        const int sz = col < R ? PADL - R + col : PADL + WZ + (col - R);
        hzl[i] = h < HZ ? (RYH + row) * LZ + sz : -1;
        const int gy = ghost(y0 + (h < HZ ? row : 0), n1);
        hzg[i] = gy * n2 + ghost(z0 + sz - PADL, n2);
    }

    // register queue along axis 0: q[s][k][R + d] = u^n(x + d) of shot s, d in [-R, R]
    vec q[S][RY][2 * R + 1];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int k = 0; k < RY; ++k)
#pragma unroll
            for (int d = 0; d < 2 * R + 1; ++d)
                q[s][k][d] = load_row<T, VZ, false, true>(
                    ucur + s * sst + (int64_t)ghost(x0 - R + d, n0) * ps + roff[k], z, n2);

    // plane-x operands, loaded one plane ahead
    vec cu[S][RY], cv[RY], chy[S][NHY1];
    avec ca[RY];
    T chz[S][NHZ];
    {
        const int64_t xo = (int64_t)x0 * ps;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
#pragma unroll
            for (int s = 0; s < S; ++s)
                cu[s][k] = load_row<T, VZ, true, false>(unew + s * sst + xo + roff[k], z, n2);
            cv[k] = load_row<T, VZ, true, false>(cc + xo + roff[k], z, n2);
            if (use_acc) ca[k] = load_row<AT, VZ, true, false>(acc + xo + roff[k], z, n2);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int i = 0; i < NHY; ++i)
                if (hyl[i] >= 0) chy[s][i] = load_row<T, VZ, false, true>(ucur + s * sst + xo + hyr[i], hyz[i], n2);
#pragma unroll
            for (int i = 0; i < NHZ; ++i) chz[s][i] = hzl[i] >= 0 ? ucur[s * sst + xo + hzg[i]] : (T)0;
        }
    }

    int e = a.blk_off[b];
    const int e_end = a.blk_off[b + 1];

    for (int x = x0; x < x1; ++x) {
        const int64_t xo = (int64_t)x * ps;
        // issue the loads of plane x + 1
        vec nq[S][RY], nu[S][RY], nv[RY], nhy[S][NHY1];
        avec na[RY];
        T nhz[S][NHZ];
        const bool more = x + 1 < x1;
        if (more) {
            const int64_t xn = xo + ps;
            const int64_t xq = (int64_t)ghost(x + 1 + R, n0) * ps;
#pragma unroll
            for (int k = 0; k < RY; ++k) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    nq[s][k] = load_row<T, VZ, false, true>(ucur + s * sst + xq + roff[k], z, n2);
                    nu[s][k] = load_row<T, VZ, true, false>(unew + s * sst + xn + roff[k], z, n2);
                }
                nv[k] = load_row<T, VZ, true, false>(cc + xn + roff[k], z, n2);
                if (use_acc) na[k] = load_row<AT, VZ, true, false>(acc + xn + roff[k], z, n2);
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
#pragma unroll
                for (int i = 0; i < NHY; ++i)
                    if (hyl[i] >= 0) nhy[s][i] = load_row<T, VZ, false, true>(ucur + s * sst + xn + hyr[i], hyz[i], n2);
#pragma unroll
                for (int i = 0; i < NHZ; ++i) nhz[s][i] = hzl[i] >= 0 ? ucur[s * sst + xn + hzg[i]] : (T)0;
            }
        }

        // stage plane x of every shot
#pragma unroll
        for (int s = 0; s < S; ++s) {
            T* L = lds + ((x & 1) * S + s) * LSZ;
#pragma unroll
            for (int k = 0; k < RY; ++k) *(vec*)(L + lofs[k]) = q[s][k][R];
#pragma unroll
            for (int i = 0; i < NHY; ++i)
                if (hyl[i] >= 0) *(vec*)(L + hyl[i]) = chy[s][i];
#pragma unroll
            for (int i = 0; i < NHZ; ++i)
                if (hzl[i] >= 0) L[hzl[i]] = chz[s][i];
        }
        __syncthreads();

        // events of this plane: [ea, e)
        const int ea = e;
        while (e < e_end && a.ev[e].plane == x) ++e;

#pragma unroll
        for (int k = 0; k < RY; ++k) {
            if (!live[k]) continue;
            const int s0 = lofs[k];
            vec un[S];
            avec an;
            const T* L0 = lds + (x & 1) * S * LSZ;
#pragma unroll
            for (int i = 0; i < VZ; ++i) {
                const T cvi = el<T, VZ>(cv[k], i);
                const T coef = a.coef_direct ? cvi : dt2 * cvi * cvi;
                AT dsum = (AT)0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const T* L = L0 + s * LSZ;
                    const T u0 = el<T, VZ>(q[s][k][R], i);
                    T lap = (T)0;
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap += w[j - 1] * ((el<T, VZ>(q[s][k][R + j], i) - u0) + (el<T, VZ>(q[s][k][R - j], i) - u0));
                    if (NDIM == 3) {
#pragma unroll
                        for (int j = 1; j <= R; ++j)
                            lap += w[j - 1] * ((L[s0 + i + j * LZ] - u0) + (L[s0 + i - j * LZ] - u0));
                    }
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap += w[j - 1] * ((L[s0 + i + j] - u0) + (L[s0 + i - j] - u0));

                    if (ea != e) {   // block-uniform: a source or receiver lies in this plane
                        T f = (T)0;
                        for (int v = ea; v < e; ++v) {
                            const Event ev = a.ev[v];
                            if (ev.lane != lane0[k] + i || ev_shot(ev.kind) != s) continue;
                            if (ev_kind(ev.kind) == EV_SRC)
                                f += ((const T*)a.wavelet)[(int64_t)a.row_src * a.nsrc + ev.idx] * (T)a.inv_vol;
                            else if (a.inject_rec)
                                f += (T)a.rec_scale * ((const T*)a.resid)[(int64_t)a.row_rec * a.nrec + ev.idx];
                        }
                        lap += f;
                    }

                    const T uni = (u0 + u0) - el<T, VZ>(cu[s][k], i) + coef * lap;
                    set_el<T, VZ>(un[s], i, uni);
                    const T d = uni - u0;
                    dsum += (AT)d * (AT)d;
                    if (a.sample && ea != e) {
                        for (int v = ea; v < e; ++v) {
                            const Event ev = a.ev[v];
                            if (ev.lane != lane0[k] + i || ev.kind != (EV_REC | (s << 1))) continue;
                            const int64_t o = (int64_t)a.row_rec * a.nrec + ev.idx;
                            if (a.traces) ((T*)a.traces)[o] = uni;
                            if (a.resid) ((T*)a.resid)[o] = uni - ((const T*)a.obs)[o];
                        }
                    }
                }
                if (use_acc) {
                    const AT ai = el<AT, VZ>(ca[k], i);
                    set_el<AT, VZ>(an, i, a.acc_sign > 0 ? ai + dsum : ai - dsum);
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s)
                __builtin_nontemporal_store(un[s], (vec*)(unew + s * sst + xo + roff[k] + z));
            if (use_acc) __builtin_nontemporal_store(an, (avec*)(acc + xo + roff[k] + z));
        }

        // rotate to plane x + 1
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
#pragma unroll
                    for (int d = 0; d < 2 * R; ++d) q[s][k][d] = q[s][k][d + 1];
                    q[s][k][2 * R] = nq[s][k];
                    cu[s][k] = nu[s][k];
                }
                cv[k] = nv[k];
                if (use_acc) ca[k] = na[k];
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
#pragma unroll
                for (int i = 0; i < NHY; ++i) chy[s][i] = nhy[s][i];
#pragma unroll
                for (int i = 0; i < NHZ; ++i) chz[s][i] = nhz[s][i];
            }
        }
    }
}

// XCD-aware logical block id: hardware block i runs on XCD i % 8, so consecutive
// logical blocks (neighbouring tiles) go to the same XCD.
__device__ __forceinline__ int logical_block(int nblk)
{
    const int per = (nblk + 7) >> 3;
    const int hb = blockIdx.x;
    return (hb & 7) * per + (hb >> 3);
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, int S>
__global__ __launch_bounds__(TZ*(TY / RY)) void step_kernel(StepArgs a)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, S> SH;
    __shared__ __attribute__((aligned(16))) T lds[SH::LDS];
    const int b = logical_block(a.nblk);
    if (b >= a.nblk) return;
    step_body<R, T, AT, NDIM, TZ, TY, RY, VZ, S>(a, b, lds);
}

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

// ---------------------------------------------------------------------------
// variants and dispatch
// ---------------------------------------------------------------------------

// (lanes along z, tile rows, rows per thread, cells per lane, largest shot group)
struct VS { int tz, ty, ry, vz, shots; };
static constexpr VS k3d[] = {
    {64, 8, 1, 1, 4}, {64, 8, 1, 2, 4}, {64, 8, 1, 4, 1}, {64, 16, 2, 2, 1},
    {64, 4, 1, 2, 1}, {64, 16, 1, 1, 1}, {64, 8, 2, 1, 1}, {64, 16, 1, 2, 1}};
static constexpr VS k2d[] = {
    {64, 1, 1, 1, 4}, {64, 1, 1, 2, 4}, {64, 1, 1, 4, 1}, {128, 1, 1, 2, 1}, {256, 1, 1, 1, 1}};

int variant_count(int ndim)
{
    return ndim == 3 ? (int)(sizeof(k3d) / sizeof(k3d[0])) : (int)(sizeof(k2d) / sizeof(k2d[0]));
}

Variant variant_shape(int ndim, int variant)
{
    Variant v{0, 0, 0, 0, 0};
    if (variant < 1 || variant > variant_count(ndim)) return v;
    const VS& s = ndim == 3 ? k3d[variant - 1] : k2d[variant - 1];
    v.tz = s.tz * s.vz;
    v.ty = s.ty;
    v.threads = s.tz * s.ty / s.ry;
    v.vz = s.vz;
    v.max_shots = s.shots;
    return v;
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, int S>
static hipError_t launch_one(int nblk, const StepArgs& a, hipStream_t s)
{
    const int grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((step_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ, S>), dim3(grid),
                       dim3(TZ * (TY / RY)), 0, s, a);
    return hipGetLastError();
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, int SMAX>
static hipError_t launch_shots(int shots, int nblk, const StepArgs& a, hipStream_t s)
{
    if (shots == 1) return launch_one<R, T, AT, NDIM, TZ, TY, RY, VZ, 1>(nblk, a, s);
    if constexpr (SMAX >= 2)
        if (shots == 2) return launch_one<R, T, AT, NDIM, TZ, TY, RY, VZ, 2>(nblk, a, s);
    if constexpr (SMAX >= 4)
        if (shots == 4) return launch_one<R, T, AT, NDIM, TZ, TY, RY, VZ, 4>(nblk, a, s);
    return hipErrorInvalidValue;
}

template <int R, typename T, typename AT>
static hipError_t launch_rt(int ndim, int variant, int shots, int nblk, const StepArgs& a, hipStream_t s)
{
    if (ndim == 3) {
        switch (variant) {
        case 1: return launch_shots<R, T, AT, 3, 64, 8, 1, 1, 4>(shots, nblk, a, s);
        case 2: return launch_shots<R, T, AT, 3, 64, 8, 1, 2, 4>(shots, nblk, a, s);
        case 3: return launch_shots<R, T, AT, 3, 64, 8, 1, 4, 1>(shots, nblk, a, s);
        case 4: return launch_shots<R, T, AT, 3, 64, 16, 2, 2, 1>(shots, nblk, a, s);
        case 5: return launch_shots<R, T, AT, 3, 64, 4, 1, 2, 1>(shots, nblk, a, s);
        case 6: return launch_shots<R, T, AT, 3, 64, 16, 1, 1, 1>(shots, nblk, a, s);
        case 7: return launch_shots<R, T, AT, 3, 64, 8, 2, 1, 1>(shots, nblk, a, s);
        case 8: return launch_shots<R, T, AT, 3, 64, 16, 1, 2, 1>(shots, nblk, a, s);
        }
    } else {
        switch (variant) {
        case 1: return launch_shots<R, T, AT, 2, 64, 1, 1, 1, 4>(shots, nblk, a, s);
        case 2: return launch_shots<R, T, AT, 2, 64, 1, 1, 2, 4>(shots, nblk, a, s);
        case 3: return launch_shots<R, T, AT, 2, 64, 1, 1, 4, 1>(shots, nblk, a, s);
        case 4: return launch_shots<R, T, AT, 2, 128, 1, 1, 2, 1>(shots, nblk, a, s);
        case 5: return launch_shots<R, T, AT, 2, 256, 1, 1, 1, 1>(shots, nblk, a, s);
        }
    }
    return hipErrorInvalidValue;
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
        }
    }
    return hipErrorInvalidValue;
}

// Resident blocks per CU the persistent grid may use: at most what the occupancy
// calculator reports and never above this cap (the dispatcher's per-CU workgroup
// limit can be lower than the wave-based occupancy for one-wave blocks).
constexpr int kPersistentBlocksPerCU = 8;

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
static hipError_t launch_persistent_one(const StepArgs* t, const int32_t* bs, int nprob, int total,
                                        int nsteps, unsigned* bar, long long timeout, hipStream_t s,
                                        int* grid_used)
{
    auto kern = step_persistent_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ>;
    const int threads = TZ * (TY / RY);
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    int grid = std::min(per_cu, kPersistentBlocksPerCU) * cus;
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
static hipError_t launch_r(int ndim, int dtype, int acc_dtype, int variant, int shots, int nblk,
                           const StepArgs& a, hipStream_t s)
{
    if (dtype == 1) return launch_rt<R, double, double>(ndim, variant, shots, nblk, a, s);
    if (acc_dtype == 1) return launch_rt<R, float, double>(ndim, variant, shots, nblk, a, s);
    return launch_rt<R, float, float>(ndim, variant, shots, nblk, a, s);
}

hipError_t launch_step(int ndim, int r, int dtype, int acc_dtype, int variant, int shots, int nblk,
                       const StepArgs& a, hipStream_t s)
{
    switch (r) {
    case 1: return launch_r<1>(ndim, dtype, acc_dtype, variant, shots, nblk, a, s);
    case 2: return launch_r<2>(ndim, dtype, acc_dtype, variant, shots, nblk, a, s);
    case 4: return launch_r<4>(ndim, dtype, acc_dtype, variant, shots, nblk, a, s);
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
