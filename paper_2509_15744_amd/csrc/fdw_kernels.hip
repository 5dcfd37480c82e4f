// HIP kernels of fdwave for gfx950 (CDNA4, wave64).
//
// The leapfrog step (paper Sec. 3.1, Eq. FDstencil2 with rho^-1 = 1, kappa = c^2,
// order-2r Laplacian) is one marching kernel for 2D and 3D grids:
//
//  * each block owns a tile of the planes normal to axis 0 (3D: TY x TZ cells of
//    axes 1 and 2; 2D: TZ cells of axis 1) and marches along axis 0 through a
//    chunk of planes;
//  * each thread keeps the 2r+1 values of its column along axis 0 in registers
//    (a rotating queue), so axis-0 neighbours are read from HBM once;
//  * the current plane is staged in LDS with an r-wide halo for the in-plane
//    neighbours (cross-shaped stencil: no corner halo);
//  * the contiguous axis maps to the 64 lanes of a wave, so every HBM access of a
//    wave is one coalesced 256-byte (f32) row segment;
//  * the new level overwrites level n-1 in place, the speed c is read instead of a
//    stored dt^2 c^2 array, and the sensitivity accumulator is updated in the same
//    pass (Alg. 1 lines 7 and 14), so a step streams four arrays;
//  * source injection, receiver sampling, the residual and the adjoint force of
//    Alg. 1 (lines 5, 6, 13) are applied by the threads that own those cells,
//    from per-block event lists sorted by plane: no separate launches per step;
//  * block ids are remapped so that consecutive tiles land on the same XCD
//    (dispatch is round-robin over the 8 XCDs) and share halo rows in its L2.
//
// Difference form of the Laplacian: sum_j w_j [(u_{+j} - u_0) + (u_{-j} - u_0)]
// keeps L applied to a constant exactly zero in f32 (rounded weights need not
// sum to zero), which removes the phase drift of the a_0 form in long runs.

#include "fdw_internal.h"

namespace fdw {

// Ghost index: half-sample mirror about the wall faces, then clamped into the
// array (the clamp only matters for tile overhang threads, which store nothing).
__device__ __forceinline__ int ghost(int i, int n)
{
    i = i < 0 ? -1 - i : i;
    i = i >= n ? 2 * n - 1 - i : i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY>
__global__ __launch_bounds__(TZ*(TY / RY)) void step_kernel(StepArgs a)
{
    constexpr int TYT = TY / RY;            // thread rows; each thread owns RY tile rows
    constexpr int NT = TZ * TYT;
    constexpr int RYH = (NDIM == 3) ? R : 0;
    constexpr int LZ = TZ + 2 * R;
    constexpr int LY = TY + 2 * RYH;
    constexpr int HALO = (NDIM == 3) ? 2 * R * TZ + 2 * R * TY : 2 * R * TY;
    __shared__ T lds[LY * LZ];

    // XCD-aware logical block id: hardware block i runs on XCD i % 8.
    const int nb = a.nblk;
    const int per = (nb + 7) >> 3;
    const int hb = blockIdx.x;
    const int b = (hb & 7) * per + (hb >> 3);
    if (b >= nb) return;
    const int tzb = b % a.ntz;
    const int rest = b / a.ntz;
    const int tyb = rest % a.nty;
    const int chb = rest / a.nty;

    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int z0 = tzb * TZ, y0 = tyb * TY;
    const int x0 = chb * a.chunk_len;
    const int x1 = min(x0 + a.chunk_len, n0);
    const int tid = threadIdx.x;
    const int lz = tid % TZ;
    const int lyt = tid / TZ;
    const int z = z0 + lz;
    const int zg = ghost(z, n2);
    const int64_t ps = (int64_t)n1 * n2;

    const T* __restrict__ ucur = (const T*)a.ucur;
    T* __restrict__ unew = (T*)a.unew;
    const T* __restrict__ cc = (const T*)a.c;
    AT* __restrict__ acc = (AT*)a.acc;
    T w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) w[j] = (T)a.w[j];
    const T dt2 = (T)a.dt2;

    int ly[RY], yg[RY];
    bool live[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        ly[k] = lyt + k * TYT;
        const int y = y0 + ly[k];
        yg[k] = ghost(y, n1);
        live[k] = (z < n2) && (y < n1);
    }

    // register queue along axis 0: q[k][R + d] = u(x + d) for d in [-R, R]
    T q[RY][2 * R + 1];
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        const int64_t col = (int64_t)yg[k] * n2 + zg;
#pragma unroll
        for (int d = 0; d < 2 * R + 1; ++d)
            q[k][d] = ucur[(int64_t)ghost(x0 - R + d, n0) * ps + col];
    }

    int e = a.blk_off[b];
    const int e_end = a.blk_off[b + 1];

    for (int x = x0; x < x1; ++x) {
        const int64_t xoff = (int64_t)x * ps;
        // stage plane x: own values from the queue, halo from memory
#pragma unroll
        for (int k = 0; k < RY; ++k) lds[(ly[k] + RYH) * LZ + lz + R] = q[k][R];
        for (int h = tid; h < HALO; h += NT) {
            int sy, sz;
            if (NDIM == 3 && h < 2 * R * TZ) {
                const int row = h / TZ;
                sz = R + h % TZ;
                sy = row < R ? row : row + TY;
            } else {
                const int hh = (NDIM == 3) ? h - 2 * R * TZ : h;
                const int row = hh / (2 * R);
                const int col = hh % (2 * R);
                sy = RYH + row;
                sz = col < R ? col : col + TZ;
            }
            const int gy = (NDIM == 3) ? ghost(y0 + sy - R, n1) : 0;
            const int gz = ghost(z0 + sz - R, n2);
            lds[sy * LZ + sz] = ucur[xoff + (int64_t)gy * n2 + gz];
        }
        __syncthreads();

        // events of this plane: [ea, e)
        const int ea = e;
        while (e < e_end && a.ev[e].plane == x) ++e;

#pragma unroll
        for (int k = 0; k < RY; ++k) {
            if (!live[k]) continue;
            const T u0 = q[k][R];
            T lap = (T)0;
#pragma unroll
            for (int j = 1; j <= R; ++j)
                lap += w[j - 1] * ((q[k][R + j] - u0) + (q[k][R - j] - u0));
            const int sy = ly[k] + RYH, sz = lz + R;
            if (NDIM == 3) {
#pragma unroll
                for (int j = 1; j <= R; ++j)
                    lap += w[j - 1] * ((lds[(sy + j) * LZ + sz] - u0) + (lds[(sy - j) * LZ + sz] - u0));
            }
#pragma unroll
            for (int j = 1; j <= R; ++j)
                lap += w[j - 1] * ((lds[sy * LZ + sz + j] - u0) + (lds[sy * LZ + sz - j] - u0));

            const int lane = ly[k] * TZ + lz;
            if (ea != e) {   // block-uniform: a source or receiver lies in this plane of the tile
                T s = (T)0;
                for (int v = ea; v < e; ++v) {
                    const Event ev = a.ev[v];
                    if (ev.lane != lane) continue;
                    if (ev.kind == EV_SRC)
                        s += ((const T*)a.wavelet)[(int64_t)a.row_src * a.nsrc + ev.idx] * (T)a.inv_vol;
                    else if (a.inject_rec)
                        s += (T)a.rec_scale * ((const T*)a.resid)[(int64_t)a.row_rec * a.nrec + ev.idx];
                }
                lap += s;
            }

            const int64_t gi = xoff + (int64_t)(y0 + ly[k]) * n2 + z;
            const T cv = cc[gi];
            const T coef = a.coef_direct ? cv : dt2 * cv * cv;
            const T um = unew[gi];
            const T un = (u0 + u0) - um + coef * lap;
            unew[gi] = un;
            if (a.acc_sign) {
                const T d = un - u0;
                const AT dd = (AT)d * (AT)d;
                acc[gi] += a.acc_sign > 0 ? dd : -dd;
            }
            if (a.sample && ea != e) {
                for (int v = ea; v < e; ++v) {
                    const Event ev = a.ev[v];
                    if (ev.lane != lane || ev.kind != EV_REC) continue;
                    const int64_t o = (int64_t)a.row_rec * a.nrec + ev.idx;
                    if (a.traces) ((T*)a.traces)[o] = un;
                    if (a.resid) ((T*)a.resid)[o] = un - ((const T*)a.obs)[o];
                }
            }
        }
        __syncthreads();

        // rotate the queue and fetch plane x + 1 + R
        const int xn = ghost(x + 1 + R, n0);
#pragma unroll
        for (int k = 0; k < RY; ++k) {
#pragma unroll
            for (int d = 0; d < 2 * R; ++d) q[k][d] = q[k][d + 1];
            q[k][2 * R] = ucur[(int64_t)xn * ps + (int64_t)yg[k] * n2 + zg];
        }
    }
}

// ---------------------------------------------------------------------------
// variants and dispatch
// ---------------------------------------------------------------------------

// 3D: (tz, ty, rows per thread); 2D: (tz, 1, 1).  Chunk lengths are chosen by the host.
struct V3 { int tz, ty, ry; };
static constexpr V3 k3d[] = {{64, 8, 2}, {64, 16, 4}, {64, 8, 1}, {64, 16, 2}, {64, 4, 1}};
static constexpr int k2d[] = {64, 128, 256};

int variant_count(int ndim)
{
    return ndim == 3 ? (int)(sizeof(k3d) / sizeof(k3d[0])) : (int)(sizeof(k2d) / sizeof(k2d[0]));
}

Variant variant_shape(int ndim, int variant)
{
    Variant v{0, 0, 0};
    if (variant < 1 || variant > variant_count(ndim)) return v;
    if (ndim == 3) {
        v.tz = k3d[variant - 1].tz;
        v.ty = k3d[variant - 1].ty;
    } else {
        v.tz = k2d[variant - 1];
        v.ty = 1;
    }
    return v;
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY>
static hipError_t launch_one(int nblk, const StepArgs& a, hipStream_t s)
{
    const int grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((step_kernel<R, T, AT, NDIM, TZ, TY, RY>), dim3(grid), dim3(TZ * (TY / RY)),
                       0, s, a);
    return hipGetLastError();
}

template <int R, typename T, typename AT>
static hipError_t launch_rt(int ndim, int variant, int nblk, const StepArgs& a, hipStream_t s)
{
    if (ndim == 3) {
        switch (variant) {
        case 1: return launch_one<R, T, AT, 3, 64, 8, 2>(nblk, a, s);
        case 2: return launch_one<R, T, AT, 3, 64, 16, 4>(nblk, a, s);
        case 3: return launch_one<R, T, AT, 3, 64, 8, 1>(nblk, a, s);
        case 4: return launch_one<R, T, AT, 3, 64, 16, 2>(nblk, a, s);
        case 5: return launch_one<R, T, AT, 3, 64, 4, 1>(nblk, a, s);
        }
    } else {
        switch (variant) {
        case 1: return launch_one<R, T, AT, 2, 64, 1, 1>(nblk, a, s);
        case 2: return launch_one<R, T, AT, 2, 128, 1, 1>(nblk, a, s);
        case 3: return launch_one<R, T, AT, 2, 256, 1, 1>(nblk, a, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int R>
static hipError_t launch_r(int ndim, int dtype, int acc_dtype, int variant, int nblk,
                           const StepArgs& a, hipStream_t s)
{
    if (dtype == 1) return launch_rt<R, double, double>(ndim, variant, nblk, a, s);
    if (acc_dtype == 1) return launch_rt<R, float, double>(ndim, variant, nblk, a, s);
    return launch_rt<R, float, float>(ndim, variant, nblk, a, s);
}

hipError_t launch_step(int ndim, int r, int dtype, int acc_dtype, int variant, int nblk,
                       const StepArgs& a, hipStream_t s)
{
    switch (r) {
    case 1: return launch_r<1>(ndim, dtype, acc_dtype, variant, nblk, a, s);
    case 2: return launch_r<2>(ndim, dtype, acc_dtype, variant, nblk, a, s);
    case 4: return launch_r<4>(ndim, dtype, acc_dtype, variant, nblk, a, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// reductions (fixed grid, fixed order: bitwise reproducible)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    return sh[0];
}

// Per block: partial sum of (x - y)^2 (x^2 when y is null) over a grid-stride range;
// optional diff output.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void sumsq_partial(const T* __restrict__ x,
                                                                const T* __restrict__ y,
                                                                T* __restrict__ diff, int64_t n,
                                                                double* __restrict__ part)
{
    __shared__ double sh[kReduceThreads];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n;
         i += (int64_t)kReduceBlocks * kReduceThreads) {
        const T d = y ? x[i] - y[i] : x[i];
        if (diff) diff[i] = d;
        s += (double)d * (double)d;
    }
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kReduceThreads) void sum_final(const double* __restrict__ part,
                                                            double* __restrict__ out)
{
    __shared__ double sh[kReduceThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < kReduceBlocks; i += kReduceThreads) s += part[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = t;
}

hipError_t launch_sum_squares(int dtype, const void* x, const void* y, void* diff_out, int64_t n,
                              double* d_part, double* d_out, hipStream_t s)
{
    if (dtype == 1)
        hipLaunchKernelGGL(sumsq_partial<double>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           (const double*)x, (const double*)y, (double*)diff_out, n, d_part);
    else
        hipLaunchKernelGGL(sumsq_partial<float>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           (const float*)x, (const float*)y, (float*)diff_out, n, d_part);
    hipLaunchKernelGGL(sum_final, dim3(1), dim3(kReduceThreads), 0, s, d_part, d_out);
    return hipGetLastError();
}

// max(c), min(c) and the count of non-finite entries: part holds 3 values per block.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void stats_partial(const T* __restrict__ c, int64_t n,
                                                                double* __restrict__ part)
{
    __shared__ double smax[kReduceThreads], smin[kReduceThreads], sbad[kReduceThreads];
    double mx = -INFINITY, mn = INFINITY, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n;
         i += (int64_t)kReduceBlocks * kReduceThreads) {
        const double v = (double)c[i];
        if (!isfinite(v)) bad += 1.0;
        else { mx = fmax(mx, v); mn = fmin(mn, v); }
    }
    const int t = threadIdx.x;
    smax[t] = mx; smin[t] = mn; sbad[t] = bad;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (t < off) {
            smax[t] = fmax(smax[t], smax[t + off]);
            smin[t] = fmin(smin[t], smin[t + off]);
            sbad[t] += sbad[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[3 * blockIdx.x + 0] = smax[0];
        part[3 * blockIdx.x + 1] = smin[0];
        part[3 * blockIdx.x + 2] = sbad[0];
    }
}

__global__ __launch_bounds__(kReduceThreads) void stats_final(const double* __restrict__ part,
                                                              double* __restrict__ out)
{
    __shared__ double smax[kReduceThreads], smin[kReduceThreads], sbad[kReduceThreads];
    double mx = -INFINITY, mn = INFINITY, bad = 0.0;
    for (int i = threadIdx.x; i < kReduceBlocks; i += kReduceThreads) {
        mx = fmax(mx, part[3 * i]);
        mn = fmin(mn, part[3 * i + 1]);
        bad += part[3 * i + 2];
    }
    const int t = threadIdx.x;
    smax[t] = mx; smin[t] = mn; sbad[t] = bad;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (t < off) {
            smax[t] = fmax(smax[t], smax[t + off]);
            smin[t] = fmin(smin[t], smin[t + off]);
            sbad[t] += sbad[t + off];
        }
        __syncthreads();
    }
    if (t == 0) { out[0] = smax[0]; out[1] = smin[0]; out[2] = sbad[0]; }
}

hipError_t launch_speed_stats(int dtype, const void* c, int64_t n, double* d_out3, double* d_part,
                              hipStream_t s)
{
    if (dtype == 1)
        hipLaunchKernelGGL(stats_partial<double>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           (const double*)c, n, d_part);
    else
        hipLaunchKernelGGL(stats_partial<float>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           (const float*)c, n, d_part);
    hipLaunchKernelGGL(stats_final, dim3(1), dim3(kReduceThreads), 0, s, d_part, d_out3);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// terminal hand-over and finalisation
// ---------------------------------------------------------------------------

// Superposed end level at the receivers: v^{nt-1} = u^{nt-1} + coef * k fdag^{nt}, and the
// kernel of the last interval, (u^nt - u^{nt-1})^2 - (v^nt - v^{nt-1})^2 (zero elsewhere, so
// the sweeps skip that interval away from the receivers).  One thread per distinct cell.
template <typename T, typename AT>
__global__ void terminal_kernel(int nuniq, const int64_t* __restrict__ ucell,
                                const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx,
                                const T* __restrict__ c, T dt2, const T* __restrict__ u_last,
                                T* __restrict__ u_prev, AT* __restrict__ acc,
                                const T* __restrict__ resid_row, T rec_scale)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nuniq) return;
    const int64_t cell = ucell[u];
    T s = (T)0;
    for (int q = uoff[u]; q < uoff[u + 1]; ++q) s += rec_scale * resid_row[uidx[q]];
    const T cv = c[cell];
    const T coef = dt2 * cv * cv;
    const T y_old = u_prev[cell];
    const T y_new = y_old + coef * s;
    const T d_old = u_last[cell] - y_old;
    const T d_new = u_last[cell] - y_new;
    acc[cell] += (AT)d_old * (AT)d_old - (AT)d_new * (AT)d_new;
    u_prev[cell] = y_new;
}

hipError_t launch_terminal(int dtype, int acc_dtype, int nuniq, const int64_t* ucell,
                           const int32_t* uoff, const int32_t* uidx, const void* c, double dt2,
                           const void* u_last, void* u_prev, void* acc, const void* resid_row,
                           double rec_scale, hipStream_t s)
{
    if (nuniq <= 0) return hipSuccess;
    const int bs = 256, gs = (nuniq + bs - 1) / bs;
    if (dtype == 1)
        hipLaunchKernelGGL((terminal_kernel<double, double>), dim3(gs), dim3(bs), 0, s, nuniq, ucell,
                           uoff, uidx, (const double*)c, dt2, (const double*)u_last,
                           (double*)u_prev, (double*)acc, (const double*)resid_row, rec_scale);
    else if (acc_dtype == 1)
        hipLaunchKernelGGL((terminal_kernel<float, double>), dim3(gs), dim3(bs), 0, s, nuniq, ucell,
                           uoff, uidx, (const float*)c, (float)dt2, (const float*)u_last,
                           (float*)u_prev, (double*)acc, (const float*)resid_row, (float)rec_scale);
    else
        hipLaunchKernelGGL((terminal_kernel<float, float>), dim3(gs), dim3(bs), 0, s, nuniq, ucell,
                           uoff, uidx, (const float*)c, (float)dt2, (const float*)u_last,
                           (float*)u_prev, (float*)acc, (const float*)resid_row, (float)rec_scale);
    return hipGetLastError();
}

// grad_c = -scale * acc / c^3, with acc = K(u,u) - K(v,v) in the sign convention
// acc = sum (u^{n+1}-u^n)^2 - sum (v^{n+1}-v^n)^2 and scale = grad_scale / k.
template <typename T, typename AT>
__global__ void finalize_kernel(int64_t n, const AT* __restrict__ acc, const T* __restrict__ c,
                                AT scale, T* __restrict__ grad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const AT cv = (AT)c[i];
        grad[i] = (T)(-scale * acc[i] / (cv * cv * cv));
    }
}

hipError_t launch_finalize(int dtype, int acc_dtype, int64_t n, const void* acc, const void* c,
                           double scale, void* grad, hipStream_t s)
{
    const int bs = 256;
    int64_t gs64 = (n + bs - 1) / bs;
    const int gs = (int)(gs64 < 65536 ? (gs64 > 0 ? gs64 : 1) : 65536);
    if (dtype == 1)
        hipLaunchKernelGGL((finalize_kernel<double, double>), dim3(gs), dim3(bs), 0, s, n,
                           (const double*)acc, (const double*)c, scale, (double*)grad);
    else if (acc_dtype == 1)
        hipLaunchKernelGGL((finalize_kernel<float, double>), dim3(gs), dim3(bs), 0, s, n,
                           (const double*)acc, (const float*)c, scale, (float*)grad);
    else
        hipLaunchKernelGGL((finalize_kernel<float, float>), dim3(gs), dim3(bs), 0, s, n,
                           (const float*)acc, (const float*)c, (float)scale, (float*)grad);
    return hipGetLastError();
}

}  // namespace fdw
