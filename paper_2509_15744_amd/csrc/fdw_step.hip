// Single-problem step kernel of fdwave: one launch per time step of one problem
// (a group of up to four shots), its kernel variants and their dispatch.  The
// per-tile work is step_body in fdw_step_body.h.

#include "fdw_step_body.h"

namespace fdw {

// Waves per SIMD the compiler is asked to make room for.  A 512-thread block puts two
// waves on each SIMD, so an instance that fits five waves per SIMD still runs only two
// blocks per CU; the f32 single-field, two-cells-per-lane instance without accumulator
// fits three blocks (six waves) without spilling.  Other instances keep the default.
template <typename T, bool ACC, int S, int VZ, int RY, int NT>
constexpr int min_waves_per_simd()
{
    return (sizeof(T) == 4 && !ACC && S == 1 && VZ == 2 && RY == 1 && NT == 512) ? 6 : 1;
}

template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, int S, bool ACC>
__global__ __launch_bounds__(TZ*(TY / RY), (min_waves_per_simd<T, ACC, S, VZ, RY, TZ*(TY / RY)>()))
void step_kernel(StepArgs a)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, S> SH;
    __shared__ __attribute__((aligned(16))) T lds[SH::LDS];
    const int b = logical_block(a.nblk);
    if (b >= a.nblk) return;
    step_body<R, T, AT, NDIM, TZ, TY, RY, VZ, S, ACC>(a, b, lds);
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
    if (a.acc_sign != 0)
        hipLaunchKernelGGL((step_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ, S, true>), dim3(grid),
                           dim3(TZ * (TY / RY)), 0, s, a);
    else
        hipLaunchKernelGGL((step_kernel<R, T, AT, NDIM, TZ, TY, RY, VZ, S, false>), dim3(grid),
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

}  // namespace fdw
