// The paper's own second-order flux-form step with variable material (Sec. 3.1, Eqs.
// FDstencil1/FDstencil2 in d dimensions), written as m u_tt - div(b grad u) = f with
// a mass coefficient m and a stiffness coefficient b per cell:
//
//   u^{n+1} = 2 u^n - u^{n-1} + (dt^2 / m) (L_b u^n + f^n)
//   (L_b u)_i = dx^-2 sum over the neighbours j of i:  h(b_i, b_j) (u_j - u_i),
//   h(p, q) = 2 p q / (p + q)                        (harmonic mean at the face)
//
// Ghost cells mirror the boundary cell and carry its material, so wall faces carry no
// flux.  The launch fuses the same per-step work as the constant-density step
// (injection, sampling, residuals) and accumulates the two kernel terms of the
// paper's gradient (Eqs. kernel1/kernel2) in discrete form:
//   * mass term: (u^{n+1} - u^n)^2 per interval, into acc (two intervals every other
//     launch, as in the constant-density sweeps);
//   * stiffness term: sum over the faces of the cell of dh/db_i (u_j - u_i)^2 for the
//     current level, with dh(p, q)/dp = 2 q^2 / (p + q)^2, into acc_b every launch;
//   * with f32 fields and f64 accumulators both terms go through f32 partial sums per
//     cell, folded into the accumulators every kPartialCycle-th accumulating launch
//     (part_mode, part_b_mode), as in the constant-density step.
//
// Layout of the work follows the constant-density step (2.5D marching along axis 0,
// three-plane register queues for u and b, the current planes of u and b staged in
// LDS with a one-cell halo, loads of plane x+1 issued before plane x is computed,
// XCD-aware block order); one wavefield per launch.

#include "fdw_aux.h"
#include "fdw_step_body.h"

namespace fdw {

// 1/x: the hardware reciprocal for f32 (within 1 ulp), an exact division for f64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// One block's share of one step.  A thread owns RY rows of the tile (rows ly,
// ly + TY / RY, ...), each with its own queues, so its loads of the next plane cover
// RY rows and fewer, larger blocks share one barrier per plane.
template <typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, bool ACC>
__device__ __forceinline__ void vd_body(const StepArgs& a, const int b, T* __restrict__ lds)
{
    typedef typename Vec<T, VZ>::type vec;
    typedef typename Vec<AT, VZ>::type avec;
    typedef typename Vec<float, VZ>::type pvec;
    static_assert(TY % RY == 0, "rows per thread divide the tile rows");
    constexpr int TYT = TY / RY;                   // thread rows
    constexpr int NT = TZ * TYT;
    constexpr int WZ = TZ * VZ;
    constexpr int RYH = (NDIM == 3) ? 1 : 0;
    constexpr int PADL = VZ;                       // one halo cell, rows kept VZ-aligned
    constexpr int LZ = PADL + WZ + PADL;
    constexpr int LSZ = (TY + 2 * RYH) * LZ;       // one plane of one field
    constexpr int HYV = (NDIM == 3) ? 2 * TZ : 0;  // halo row vectors above and below
    constexpr int HZ = 2 * TY;                     // halo cells left and right
    constexpr int NHY = (HYV + NT - 1) / NT;
    constexpr int NHZ = (HZ + NT - 1) / NT;
    constexpr int NHY1 = NHY > 0 ? NHY : 1;

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
    const int z = z0 + lz * VZ;
    const int pitch = a.pitch;                  // row stride (rows may be padded)
    const int64_t ps = (int64_t)n1 * pitch;
    int roff[RY], lofs[RY], lane0[RY];
    bool live[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        const int ly = lyt + k * TYT;
        const int y = y0 + ly;
        live[k] = z < n2 && y < n1;
        roff[k] = ghost(y, n1) * pitch;
        lofs[k] = (ly + RYH) * LZ + PADL + lz * VZ;
        lane0[k] = ly * WZ + lz * VZ;
    }

    const GLOBAL_AS T* __restrict__ ucur = (const GLOBAL_AS T*)a.ucur;
    GLOBAL_AS T* __restrict__ unew = (GLOBAL_AS T*)a.unew;
    const GLOBAL_AS T* __restrict__ mass = (const GLOBAL_AS T*)a.c;
    const GLOBAL_AS T* __restrict__ stiff = (const GLOBAL_AS T*)a.stiff;
    GLOBAL_AS AT* __restrict__ acc = (GLOBAL_AS AT*)a.acc;
    GLOBAL_AS AT* __restrict__ accb = (GLOBAL_AS AT*)a.acc_b;
    const bool use_acc = ACC && a.acc_sign != 0;
    const bool use_accb = ACC && a.acc_face != 0;
    // f32 partial sums of both kernel terms (f32 fields with f64 accumulators): what each
    // accumulating launch reads and writes (modes as in the constant-density step)
    constexpr bool PARTS = ACC && sizeof(T) == 4 && sizeof(AT) == 8;
    GLOBAL_AS float* __restrict__ part = (GLOBAL_AS float*)a.part;
    GLOBAL_AS float* __restrict__ partb = (GLOBAL_AS float*)a.part_b;
    const int pm = (PARTS && use_acc) ? a.part_mode : PM_DIRECT;
    const int pmb = (PARTS && use_accb) ? a.part_b_mode : PM_DIRECT;
    const bool rd_acc = use_acc && (pm == PM_DIRECT || pm == PM_FLUSH);
    const bool rd_part = PARTS && use_acc && (pm == PM_ADD || pm == PM_FLUSH);
    const bool wr_part = PARTS && use_acc && (pm == PM_START || pm == PM_ADD);
    const bool rd_accb = use_accb && (pmb == PM_DIRECT || pmb == PM_FLUSH);
    const bool rd_partb = PARTS && use_accb && (pmb == PM_ADD || pmb == PM_FLUSH);
    const bool wr_partb = PARTS && use_accb && (pmb == PM_START || pmb == PM_ADD);
    const T inv_dx2 = (T)a.w[0];
    const T dt2 = (T)a.dt2;

    // halo rows (3D) and halo columns: LDS slot and in-plane offset
    int hyl[NHY1], hyr[NHY1], hyz[NHY1];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int h = tid + i * NT;
        const int row = h / TZ;                   // 0: the row above the tile, 1: below
        const int sy = row < 1 ? 0 : TY + 1;
        const int cz = (h % TZ) * VZ;
        hyl[i] = h < HYV ? sy * LZ + PADL + cz : -1;
        hyr[i] = ghost(y0 + sy - 1, n1) * pitch;
        hyz[i] = z0 + cz;
    }
    int hzl[NHZ], hzg[NHZ];
#pragma unroll
    for (int i = 0; i < NHZ; ++i) {
        const int h = tid + i * NT;
        const int row = h / 2;
        const int sz = (h % 2) == 0 ? PADL - 1 : PADL + WZ;
        hzl[i] = h < HZ ? (RYH + row) * LZ + sz : -1;
        hzg[i] = ghost(y0 + (h < HZ ? row : 0), n1) * pitch + ghost(z0 + sz - PADL, n2);
    }

    // register queues along axis 0: planes x-1, x, x+1 of u^n and of b, per own row
    vec qu[RY][3], qb[RY][3];
#pragma unroll
    for (int k = 0; k < RY; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t xo = (int64_t)ghost(x0 - 1 + d, n0) * ps + roff[k];
            qu[k][d] = load_row<T, VZ, false, true>(ucur + xo, z, n2);
            qb[k][d] = load_row<T, VZ, false, true>(stiff + xo, z, n2);
        }
    // plane-x operands, loaded one plane ahead
    vec cu[RY], cm[RY], chyu[NHY1], chyb[NHY1];
    avec ca[RY], cab[RY];
    pvec cp[RY], cpb[RY];
    T chzu[NHZ], chzb[NHZ];
    {
        const int64_t xo = (int64_t)x0 * ps;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            cu[k] = load_row<T, VZ, true, false>(unew + xo + roff[k], z, n2);
            cm[k] = load_row<T, VZ, true, false>(mass + xo + roff[k], z, n2);
            if (rd_acc) ca[k] = load_row<AT, VZ, true, false>(acc + xo + roff[k], z, n2);
            if (rd_accb) cab[k] = load_row<AT, VZ, true, false>(accb + xo + roff[k], z, n2);
            if (rd_part) cp[k] = load_row<float, VZ, true, false>(part + xo + roff[k], z, n2);
            if (rd_partb) cpb[k] = load_row<float, VZ, true, false>(partb + xo + roff[k], z, n2);
        }
#pragma unroll
        for (int i = 0; i < NHY; ++i)
            if (hyl[i] >= 0) {
                chyu[i] = load_row<T, VZ, false, true>(ucur + xo + hyr[i], hyz[i], n2);
                chyb[i] = load_row<T, VZ, false, true>(stiff + xo + hyr[i], hyz[i], n2);
            }
#pragma unroll
        for (int i = 0; i < NHZ; ++i) {
            chzu[i] = hzl[i] >= 0 ? ucur[xo + hzg[i]] : (T)0;
            chzb[i] = hzl[i] >= 0 ? stiff[xo + hzg[i]] : (T)0;
        }
    }

    __shared__ EventStage<T> est;
    PlaneEvents pe;
    events_begin(pe, a, b);

    for (int x = x0; x < x1; ++x) {
        const int64_t xo = (int64_t)x * ps;
        // issue the loads of plane x + 1
        vec nqu[RY], nqb[RY], ncu[RY], ncm[RY], nhyu[NHY1], nhyb[NHY1];
        avec nca[RY], ncab[RY];
        pvec ncp[RY], ncpb[RY];
        T nhzu[NHZ], nhzb[NHZ];
        const bool more = x + 1 < x1;
        if (more) {
            const int64_t xn = xo + ps;
            const int64_t xq = (int64_t)ghost(x + 2, n0) * ps;
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                nqu[k] = load_row<T, VZ, false, true>(ucur + xq + roff[k], z, n2);
                nqb[k] = load_row<T, VZ, false, true>(stiff + xq + roff[k], z, n2);
                ncu[k] = load_row<T, VZ, true, false>(unew + xn + roff[k], z, n2);
                ncm[k] = load_row<T, VZ, true, false>(mass + xn + roff[k], z, n2);
                if (rd_acc) nca[k] = load_row<AT, VZ, true, false>(acc + xn + roff[k], z, n2);
                if (rd_accb) ncab[k] = load_row<AT, VZ, true, false>(accb + xn + roff[k], z, n2);
                if (rd_part) ncp[k] = load_row<float, VZ, true, false>(part + xn + roff[k], z, n2);
                if (rd_partb) ncpb[k] = load_row<float, VZ, true, false>(partb + xn + roff[k], z, n2);
            }
#pragma unroll
            for (int i = 0; i < NHY; ++i)
                if (hyl[i] >= 0) {
                    nhyu[i] = load_row<T, VZ, false, true>(ucur + xn + hyr[i], hyz[i], n2);
                    nhyb[i] = load_row<T, VZ, false, true>(stiff + xn + hyr[i], hyz[i], n2);
                }
#pragma unroll
            for (int i = 0; i < NHZ; ++i) {
                nhzu[i] = hzl[i] >= 0 ? ucur[xn + hzg[i]] : (T)0;
                nhzb[i] = hzl[i] >= 0 ? stiff[xn + hzg[i]] : (T)0;
            }
        }

        // stage plane x of u and of b
        T* Lu = lds + (x & 1) * 2 * LSZ;
        T* Lb = Lu + LSZ;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            *(vec*)(Lu + lofs[k]) = qu[k][1];
            *(vec*)(Lb + lofs[k]) = qb[k][1];
        }
#pragma unroll
        for (int i = 0; i < NHY; ++i)
            if (hyl[i] >= 0) {
                *(vec*)(Lu + hyl[i]) = chyu[i];
                *(vec*)(Lb + hyl[i]) = chyb[i];
            }
#pragma unroll
        for (int i = 0; i < NHZ; ++i)
            if (hzl[i] >= 0) {
                Lu[hzl[i]] = chzu[i];
                Lb[hzl[i]] = chzb[i];
            }
        events_at_plane<T, NT>(pe, a, est, x, tid);
        __syncthreads();

#pragma unroll
        for (int k = 0; k < RY; ++k) {
            if (!live[k]) continue;
            const int lo = lofs[k];
            vec un;
            avec an, abn;
            pvec pn, pbn;
#pragma unroll
            for (int i = 0; i < VZ; ++i) {
                const T u0 = el<T, VZ>(qu[k][1], i);
                const T b0 = el<T, VZ>(qb[k][1], i);
                T lap = (T)0;
                T fb = (T)0;   // this level's stiffness terms, added to the accumulator in AT
                auto face = [&](T uj, T bj) {
                    // with t = b_j / (b_0 + b_j): h = 2 b_0 t, dh/db_0 = 2 t^2
                    const T t = bj * recip(b0 + bj);
                    const T d = uj - u0;
                    lap += (b0 * (t + t)) * d;
                    if (use_accb) fb += ((t + t) * t) * (d * d);
                };
                face(el<T, VZ>(qu[k][0], i), el<T, VZ>(qb[k][0], i));
                face(el<T, VZ>(qu[k][2], i), el<T, VZ>(qb[k][2], i));
                if (NDIM == 3) {
                    face(Lu[lo + i - LZ], Lb[lo + i - LZ]);
                    face(Lu[lo + i + LZ], Lb[lo + i + LZ]);
                }
                face(Lu[lo + i - 1], Lb[lo + i - 1]);
                face(Lu[lo + i + 1], Lb[lo + i + 1]);
                lap *= inv_dx2;
                if (pe.has) lap += point_force<false>(pe, a, est, lane0[k] + i, 0);
                const T cui = el<T, VZ>(cu[k], i);
                const T coef = dt2 * recip(el<T, VZ>(cm[k], i));
                const T uni = (u0 + u0) - cui + coef * lap;
                set_el<T, VZ>(un, i, uni);
                if (a.sample && pe.has) sample_receivers<false>(pe, a, est, lane0[k] + i, 0, uni);
                if (use_acc) {
                    const AT d = (AT)(uni - u0);
                    const AT dp = a.acc_prev ? (AT)(u0 - cui) : (AT)0;
                    const AT dsum = d * d + dp * dp;
                    const AT tot = rd_part ? dsum + (AT)el<float, VZ>(cp[k], i) : dsum;
                    if (rd_acc) {
                        const AT ai = el<AT, VZ>(ca[k], i);
                        set_el<AT, VZ>(an, i, a.acc_sign > 0 ? ai + tot : ai - tot);
                    }
                    if (wr_part) set_el<float, VZ>(pn, i, (float)tot);
                }
                if (use_accb) {
                    const AT totb = rd_partb ? (AT)fb + (AT)el<float, VZ>(cpb[k], i) : (AT)fb;
                    if (rd_accb) {
                        const AT bi = el<AT, VZ>(cab[k], i);
                        set_el<AT, VZ>(abn, i, a.acc_face > 0 ? bi + totb : bi - totb);
                    }
                    if (wr_partb) set_el<float, VZ>(pbn, i, (float)totb);
                }
            }
            const int64_t o = xo + roff[k] + z;
            __builtin_nontemporal_store(un, (vec*)(unew + o));
            if (rd_acc) __builtin_nontemporal_store(an, (avec*)(acc + o));
            if (rd_accb) __builtin_nontemporal_store(abn, (avec*)(accb + o));
            if (wr_part) __builtin_nontemporal_store(pn, (pvec*)(part + o));
            if (wr_partb) __builtin_nontemporal_store(pbn, (pvec*)(partb + o));
        }

        // rotate to plane x + 1
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                qu[k][0] = qu[k][1]; qu[k][1] = qu[k][2]; qu[k][2] = nqu[k];
                qb[k][0] = qb[k][1]; qb[k][1] = qb[k][2]; qb[k][2] = nqb[k];
                cu[k] = ncu[k];
                cm[k] = ncm[k];
                if (rd_acc) ca[k] = nca[k];
                if (rd_accb) cab[k] = ncab[k];
                if (rd_part) cp[k] = ncp[k];
                if (rd_partb) cpb[k] = ncpb[k];
            }
#pragma unroll
            for (int i = 0; i < NHY; ++i) { chyu[i] = nhyu[i]; chyb[i] = nhyb[i]; }
#pragma unroll
            for (int i = 0; i < NHZ; ++i) { chzu[i] = nhzu[i]; chzb[i] = nhzb[i]; }
        }
    }
}

template <typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, bool ACC>
__global__ __launch_bounds__(TZ * (TY / RY)) void vd_step_kernel(StepArgs a)
{
    constexpr int LZ = 2 * VZ + TZ * VZ;
    constexpr int LSZ = (TY + ((NDIM == 3) ? 2 : 0)) * LZ;
    __shared__ __attribute__((aligned(16))) T lds[2 * 2 * LSZ];
    const int b = logical_block(a.nblk);
    if (b >= a.nblk) return;
    vd_body<T, AT, NDIM, TZ, TY, RY, VZ, ACC>(a, b, lds);
}

template <typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ>
static hipError_t launch_vd_one(int nblk, const StepArgs& a, hipStream_t s)
{
    const int grid = ((nblk + 7) / 8) * 8;
    if (a.acc_sign != 0 || a.acc_face != 0)
        hipLaunchKernelGGL((vd_step_kernel<T, AT, NDIM, TZ, TY, RY, VZ, true>), dim3(grid),
                           dim3(TZ * (TY / RY)), 0, s, a);
    else
        hipLaunchKernelGGL((vd_step_kernel<T, AT, NDIM, TZ, TY, RY, VZ, false>), dim3(grid),
                           dim3(TZ * (TY / RY)), 0, s, a);
    return hipGetLastError();
}

// The tile shapes of the step variants (3D: 1 and 2, one or two cells per lane, 5, a
// 64 x 4 tile with two cells per lane, and 7, a 64 x 8 tile with two rows per thread;
// 2D also 4 and 5, rows of 128 x 2 and 256 cells, which keep more waves resident per
// block than one 64-lane wavefront), so the block decomposition and event lists of a
// plan serve both kernels.
template <typename T, typename AT>
static hipError_t launch_vd_rt(int ndim, int variant, int nblk, const StepArgs& a, hipStream_t s)
{
    if (ndim == 3) {
        if (variant == 1) return launch_vd_one<T, AT, 3, 64, 8, 1, 1>(nblk, a, s);
        if (variant == 2) return launch_vd_one<T, AT, 3, 64, 8, 1, 2>(nblk, a, s);
        if (variant == 5) return launch_vd_one<T, AT, 3, 64, 4, 1, 2>(nblk, a, s);
        if (variant == 7) return launch_vd_one<T, AT, 3, 64, 8, 2, 1>(nblk, a, s);
    } else {
        if (variant == 1) return launch_vd_one<T, AT, 2, 64, 1, 1, 1>(nblk, a, s);
        if (variant == 2) return launch_vd_one<T, AT, 2, 64, 1, 1, 2>(nblk, a, s);
        if (variant == 4) return launch_vd_one<T, AT, 2, 128, 1, 1, 2>(nblk, a, s);
        if (variant == 5) return launch_vd_one<T, AT, 2, 256, 1, 1, 1>(nblk, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_vd_step(int ndim, int dtype, int acc_dtype, int variant, int nblk, const StepArgs& a,
                          hipStream_t s)
{
    if (dtype == 1) return launch_vd_rt<double, double>(ndim, variant, nblk, a, s);
    if (acc_dtype == 1) return launch_vd_rt<float, double>(ndim, variant, nblk, a, s);
    return launch_vd_rt<float, float>(ndim, variant, nblk, a, s);
}

// ---------------------------------------------------------------------------
// stability bound of the variable-material scheme
// ---------------------------------------------------------------------------

// Per cell, the Gershgorin row sum of the symmetric form M^-1/2 K M^-1/2 of the
// spatial operator (times dx^2):
//   s_i = sum over the interior faces f of cell i of h_f (1/m_i + 1/sqrt(m_i m_j)),
// h_f the harmonic-mean face stiffness; wall faces carry no flux and add nothing.
// Partial maxima per block in f64 (n1 = 1 for 2D grids).
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void vd_bound_partial(const T* __restrict__ m,
                                                                   const T* __restrict__ b, int64_t n0,
                                                                   int64_t n1, int64_t n2,
                                                                   double* __restrict__ part)
{
    __shared__ double smax[kReduceThreads];
    const int64_t ncell = n0 * n1 * n2;
    const int64_t strides[3] = {n1 * n2, n2, 1};
    const int64_t ext[3] = {n0, n1, n2};
    double mx = 0.0;
    for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < ncell;
         cell += (int64_t)gridDim.x * blockDim.x) {
        const int64_t idx[3] = {cell / strides[0], (cell / n2) % n1, cell % n2};
        const double mi = (double)m[cell];
        const double bi = (double)b[cell];
        double sum = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            for (int dir = -1; dir <= 1; dir += 2) {
                const int64_t q = idx[ax] + dir;
                if (q < 0 || q >= ext[ax]) continue;
                const int64_t j = cell + dir * strides[ax];
                const double mj = (double)m[j];
                const double bj = (double)b[j];
                const double h = 2.0 * bi * bj / (bi + bj);
                sum += h * (1.0 / mi + 1.0 / sqrt(mi * mj));
            }
        }
        mx = fmax(mx, sum);
    }
    const int t = threadIdx.x;
    smax[t] = mx;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (t < off) smax[t] = fmax(smax[t], smax[t + off]);
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = smax[0];
}

__global__ __launch_bounds__(kReduceThreads) void max_final(const double* __restrict__ part, int nparts,
                                                            double* __restrict__ out)
{
    __shared__ double smax[kReduceThreads];
    double mx = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kReduceThreads) mx = fmax(mx, part[i]);
    const int t = threadIdx.x;
    smax[t] = mx;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (t < off) smax[t] = fmax(smax[t], smax[t + off]);
        __syncthreads();
    }
    if (t == 0) out[0] = smax[0];
}

hipError_t launch_vd_bound(int dtype, const void* m, const void* b, int64_t n0, int64_t n1, int64_t n2,
                           double* d_out, double* d_part, hipStream_t s)
{
    if (dtype == 1)
        hipLaunchKernelGGL(vd_bound_partial<double>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           (const double*)m, (const double*)b, n0, n1, n2, d_part);
    else
        hipLaunchKernelGGL(vd_bound_partial<float>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           (const float*)m, (const float*)b, n0, n1, n2, d_part);
    hipLaunchKernelGGL(max_final, dim3(1), dim3(kReduceThreads), 0, s, (const double*)d_part, kReduceBlocks,
                       d_out);
    return hipGetLastError();
}

}  // namespace fdw
