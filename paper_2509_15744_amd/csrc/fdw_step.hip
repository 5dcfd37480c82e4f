// The fused leapfrog step of fdwave for gfx950 (CDNA4, wave64).
//
// One step of the scheme (paper Sec. 3.1, Eq. FDstencil2 with rho^-1 = 1,
// kappa = c^2, order-2r Laplacian) over the whole grid, fused with the work that
// Alg. 1 does per time step: source injection (line 4), receiver sampling, the
// residual / adjoint force (line 5) and the kernel increments K(u,u) (line 7) or
// K(v,v) (line 14).  One launch per time step; 2D and 3D share the code.
//
// Layout of the work:
//  * a block owns a tile of the planes normal to axis 0 (3D: TY x TZ cells of
//    axes 1 and 2; 2D: TZ cells of axis 1) and marches along axis 0 through a
//    chunk of planes;
//  * each thread keeps the 2r+1 values of its column along axis 0 in registers
//    (a rotating queue), so axis-0 neighbours cost no extra reads;
//  * the current plane is staged in LDS with an r-wide halo for the in-plane
//    neighbours (cross-shaped stencil: no corner halo), double-buffered so one
//    barrier per plane suffices;
//  * software pipelining: every load of plane x+1 (queue entry x+1+r, halo,
//    u^{n-1}, c, accumulator) is issued before plane x is computed, so a whole
//    plane of work covers the memory latency;
//  * the contiguous axis maps to the 64 lanes of a wave: every access of a wave
//    is one coalesced row segment; plane bases are wave-uniform 64-bit pointers
//    and in-plane offsets 32-bit;
//  * u^{n+1} overwrites u^{n-1} in place and the speed c is read instead of a
//    stored dt^2 c^2 array, so a step streams four arrays; those streams are read
//    and written non-temporally, which leaves the cache to the u^n halos;
//  * block ids are remapped so that consecutive tiles run on the same XCD
//    (dispatch is round-robin over the 8 XCDs) and share halo rows in its L2.
//
// Difference form of the Laplacian, sum_j w_j [(u_{+j} - u_0) + (u_{-j} - u_0)]:
// L applied to a constant is exactly zero in f32 even though the rounded weights
// do not sum to zero, which removes the phase drift of the a_0 form.

#include "fdw_internal.h"

namespace fdw {

// Ghost index: half-sample mirror about the wall faces, then clamped into the
// array (the clamp only matters for tile-overhang threads, which store nothing).
__device__ __forceinline__ int ghost(int i, int n)
{
    i = i < 0 ? -1 - i : i;
    i = i >= n ? 2 * n - 1 - i : i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T v, T* p) { __builtin_nontemporal_store(v, p); }

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY>
__global__ __launch_bounds__(TZ*(TY / RY)) void step_kernel(StepArgs a)
{
    constexpr int TYT = TY / RY;            // thread rows; a thread owns RY tile rows
    constexpr int NT = TZ * TYT;
    constexpr int RYH = (NDIM == 3) ? R : 0;
    constexpr int LZ = TZ + 2 * R;
    constexpr int LSZ = (TY + 2 * RYH) * LZ;
    constexpr int HY = (NDIM == 3) ? 2 * R * TZ : 0;   // halo rows above and below
    constexpr int HALO = HY + 2 * R * TY;              // plus halo columns left and right
    constexpr int NH = (HALO + NT - 1) / NT;           // halo cells per thread
    __shared__ T lds[2][LSZ];

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
    const bool use_acc = a.acc_sign != 0;
    T w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) w[j] = (T)a.w[j];
    const T dt2 = (T)a.dt2;

    // own cells: in-plane offset (ghosted for overhang threads, which never store)
    int off[RY], lofs[RY], lane[RY];
    bool live[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        const int ly = lyt + k * TYT;
        const int y = y0 + ly;
        off[k] = ghost(y, n1) * n2 + zg;
        live[k] = (z < n2) && (y < n1);
        lofs[k] = (ly + RYH) * LZ + lz + R;
        lane[k] = ly * TZ + lz;
    }
    // halo cells of this thread: LDS slot and in-plane source offset
    int hl[NH], hg[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int h = tid + i * NT;
        int sy = 0, sz = 0;
        if (h < HY) {
            const int row = h / TZ;
            sz = R + h % TZ;
            sy = row < R ? row : row + TY;
        } else {
            const int hh = h - HY;
            sy = RYH + hh / (2 * R);
            const int col = hh % (2 * R);
            sz = col < R ? col : col + TZ;
        }
        hl[i] = h < HALO ? sy * LZ + sz : -1;
        const int gy = (NDIM == 3) ? ghost(y0 + sy - R, n1) : 0;
        hg[i] = gy * n2 + ghost(z0 + sz - R, n2);
    }

    // register queue along axis 0: q[k][R + d] = u^n(x + d), d in [-R, R]
    T q[RY][2 * R + 1];
#pragma unroll
    for (int k = 0; k < RY; ++k)
#pragma unroll
        for (int d = 0; d < 2 * R + 1; ++d)
            q[k][d] = ucur[(int64_t)ghost(x0 - R + d, n0) * ps + off[k]];

    // plane-x operands, loaded one plane ahead
    T cu[RY], cv[RY], ch[NH];
    AT ca[RY];
    {
        const int64_t xo = (int64_t)x0 * ps;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            cu[k] = ld_stream(unew + xo + off[k]);
            cv[k] = ld_stream(cc + xo + off[k]);
            ca[k] = use_acc ? ld_stream(acc + xo + off[k]) : (AT)0;
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) ch[i] = hl[i] >= 0 ? ucur[xo + hg[i]] : (T)0;
    }

    int e = a.blk_off[b];
    const int e_end = a.blk_off[b + 1];

    for (int x = x0; x < x1; ++x) {
        const int64_t xo = (int64_t)x * ps;
        // issue the loads of plane x + 1
        T nq[RY], nu[RY], nv[RY], nh[NH];
        AT na[RY];
        const bool more = x + 1 < x1;
        if (more) {
            const int64_t xn = xo + ps;
            const int64_t xq = (int64_t)ghost(x + 1 + R, n0) * ps;
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                nq[k] = ucur[xq + off[k]];
                nu[k] = ld_stream(unew + xn + off[k]);
                nv[k] = ld_stream(cc + xn + off[k]);
                na[k] = use_acc ? ld_stream(acc + xn + off[k]) : (AT)0;
            }
#pragma unroll
            for (int i = 0; i < NH; ++i) nh[i] = hl[i] >= 0 ? ucur[xn + hg[i]] : (T)0;
        }

        // stage plane x
        T* L = lds[x & 1];
#pragma unroll
        for (int k = 0; k < RY; ++k) L[lofs[k]] = q[k][R];
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (hl[i] >= 0) L[hl[i]] = ch[i];
        __syncthreads();

        // events of this plane: [ea, e)
        const int ea = e;
        while (e < e_end && a.ev[e].plane == x) ++e;

#pragma unroll
        for (int k = 0; k < RY; ++k) {
            if (!live[k]) continue;
            const T u0 = q[k][R];
            const int s0 = lofs[k];
            T lap = (T)0;
#pragma unroll
            for (int j = 1; j <= R; ++j)
                lap += w[j - 1] * ((q[k][R + j] - u0) + (q[k][R - j] - u0));
            if (NDIM == 3) {
#pragma unroll
                for (int j = 1; j <= R; ++j)
                    lap += w[j - 1] * ((L[s0 + j * LZ] - u0) + (L[s0 - j * LZ] - u0));
            }
#pragma unroll
            for (int j = 1; j <= R; ++j)
                lap += w[j - 1] * ((L[s0 + j] - u0) + (L[s0 - j] - u0));

            if (ea != e) {   // block-uniform: a source or receiver lies in this plane of the tile
                T s = (T)0;
                for (int v = ea; v < e; ++v) {
                    const Event ev = a.ev[v];
                    if (ev.lane != lane[k]) continue;
                    if (ev.kind == EV_SRC)
                        s += ((const T*)a.wavelet)[(int64_t)a.row_src * a.nsrc + ev.idx] * (T)a.inv_vol;
                    else if (a.inject_rec)
                        s += (T)a.rec_scale * ((const T*)a.resid)[(int64_t)a.row_rec * a.nrec + ev.idx];
                }
                lap += s;
            }

            const T coef = a.coef_direct ? cv[k] : dt2 * cv[k] * cv[k];
            const T un = (u0 + u0) - cu[k] + coef * lap;
            st_stream(un, unew + xo + off[k]);
            if (use_acc) {
                const T d = un - u0;
                const AT dd = (AT)d * (AT)d;
                st_stream(a.acc_sign > 0 ? ca[k] + dd : ca[k] - dd, acc + xo + off[k]);
            }
            if (a.sample && ea != e) {
                for (int v = ea; v < e; ++v) {
                    const Event ev = a.ev[v];
                    if (ev.lane != lane[k] || ev.kind != EV_REC) continue;
                    const int64_t o = (int64_t)a.row_rec * a.nrec + ev.idx;
                    if (a.traces) ((T*)a.traces)[o] = un;
                    if (a.resid) ((T*)a.resid)[o] = un - ((const T*)a.obs)[o];
                }
            }
        }

        // rotate to plane x + 1
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
#pragma unroll
                for (int d = 0; d < 2 * R; ++d) q[k][d] = q[k][d + 1];
                q[k][2 * R] = nq[k];
                cu[k] = nu[k];
                cv[k] = nv[k];
                ca[k] = na[k];
            }
#pragma unroll
            for (int i = 0; i < NH; ++i) ch[i] = nh[i];
        }
    }
}

// ---------------------------------------------------------------------------
// variants and dispatch
// ---------------------------------------------------------------------------

// 3D: (tz, ty, rows per thread); 2D: tz.  Chunk lengths are chosen by the host.
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
        v.threads = v.tz * v.ty / k3d[variant - 1].ry;
    } else {
        v.tz = k2d[variant - 1];
        v.ty = 1;
        v.threads = v.tz;
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

}  // namespace fdw
