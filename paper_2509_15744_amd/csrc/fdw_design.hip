// Kernels around the sweeps of gradient-based design (the topology-optimisation chain
// of Sec. 2.3 and the update of Eq. gradientdescent with Adam):
//
//  * design_map: design field gamma on a box of cells -> density filter with linear
//    decay (weights r_f - |x|, normalised by their sum over the neighbours inside the
//    box) -> smoothed Heaviside projection (threshold eta, sharpness beta) -> clip to
//    [lo, hi] -> material m, b affine in the result (rho-scaling of Eq.
//    scalarwaveequation and the linear inverse-density / inverse-bulk-modulus maps of
//    Eq. wavetopopt are both affine);
//  * design_adjoint: dC/dgamma from dC/dm and dC/db by the chain rule of that map: the
//    per-cell factors (material slope, clip mask, projection slope, 1 / weight sum) in
//    one pass, then the filter's transpose (the same symmetric neighbourhood sum) in a
//    second;
//  * adam: the Adam update (bias-corrected first and second moments) followed by the
//    clip of the design field to its admissible interval.
//
// All three stream over the design box once or twice; they run once per design
// iteration, next to the 2 nt stencil launches of the sweeps.
#include <hip/hip_runtime.h>

#include "fdw_aux.h"

namespace fdw {

namespace {

constexpr int kThreads = 256;

__device__ inline void box_coords(const DesignArgs& d, int64_t i, int64_t q[3])
{
    q[2] = i % d.e[2];
    const int64_t r = i / d.e[2];
    q[1] = r % d.e[1];
    q[0] = r / d.e[1];
}

__device__ inline int64_t grid_cell(const DesignArgs& d, const int64_t q[3])
{
    return ((d.o[0] + q[0]) * d.n[1] + (d.o[1] + q[1])) * d.n[2] + (d.o[2] + q[2]);
}

// sum_k w_k x_k and sum_k w_k over the box cells k with |x_k - x_q| < rf,
// w_k = rf - |x_k - x_q| (offsets in cells).
template <typename T>
__device__ inline void neighbourhood_sum(const DesignArgs& d, const T* __restrict__ x, const int64_t q[3],
                                         T& sx, T& sw)
{
    int lo[3], hi[3];
    for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = -(int)(q[ax] < d.R ? q[ax] : d.R);
        const int64_t up = d.e[ax] - 1 - q[ax];
        hi[ax] = (int)(up < d.R ? up : d.R);
    }
    const T rf = (T)d.rf;
    sx = (T)0;
    sw = (T)0;
    for (int a = lo[0]; a <= hi[0]; ++a) {
        for (int c = lo[1]; c <= hi[1]; ++c) {
            const int64_t row = ((q[0] + a) * d.e[1] + (q[1] + c)) * d.e[2] + q[2];
            for (int z = lo[2]; z <= hi[2]; ++z) {
                const T w = rf - sqrt((T)(a * a + c * c + z * z));
                if (w <= (T)0) continue;
                sx += w * x[row + z];
                sw += w;
            }
        }
    }
}

// Projection and its slope: h = (th0 + tanh(beta (gt - eta))) / hnorm,
// dh/dgt = beta (1 - tanh^2) / hnorm; identity without projection.
template <typename T>
__device__ inline T project(const DesignArgs& d, T gt, T* slope)
{
    if (!d.proj) {
        *slope = (T)1;
        return gt;
    }
    const T t = tanh((T)d.beta * (gt - (T)d.eta));
    *slope = (T)d.beta * ((T)1 - t * t) / (T)d.hnorm;
    return ((T)d.th0 + t) / (T)d.hnorm;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void design_map_kernel(DesignArgs d, const T* __restrict__ gamma,
                                                              T* __restrict__ m, T* __restrict__ b,
                                                              T* __restrict__ gbar)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.nbox;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t q[3];
        box_coords(d, i, q);
        T sx, sw;
        neighbourhood_sum(d, gamma, q, sx, sw);
        T slope;
        T h = project(d, sx / sw, &slope);
        const T lo = (T)d.lo, hi = (T)d.hi;
        h = h < lo ? lo : (h > hi ? hi : h);   // NaN passes through
        if (gbar) gbar[i] = h;
        const int64_t cell = grid_cell(d, q);
        m[cell] = (T)d.m0 + h * (T)d.dm;
        b[cell] = (T)d.b0 + h * (T)d.db;
    }
}

// First adjoint pass: t_i = (gm dm + gb db) [lo <= h_i <= hi] (dh/dgt)_i / sum_k w_ik.
template <typename T>
__global__ __launch_bounds__(kThreads) void design_adjoint_cells(DesignArgs d, const T* __restrict__ gamma,
                                                                 const T* __restrict__ grad_m,
                                                                 const T* __restrict__ grad_b,
                                                                 T* __restrict__ t)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.nbox;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t q[3];
        box_coords(d, i, q);
        T sx, sw;
        neighbourhood_sum(d, gamma, q, sx, sw);
        T slope;
        const T h = project(d, sx / sw, &slope);
        const bool inside = (T)d.lo <= h && h <= (T)d.hi;
        const int64_t cell = grid_cell(d, q);
        const T g = grad_m[cell] * (T)d.dm + grad_b[cell] * (T)d.db;
        t[i] = inside ? g * slope / sw : (T)0;
    }
}

// Second adjoint pass: dC/dgamma_k = sum_i w_ik t_i (the filter weights are symmetric
// and so is the neighbourhood relation inside the box).
template <typename T>
__global__ __launch_bounds__(kThreads) void design_adjoint_filter(DesignArgs d, const T* __restrict__ t,
                                                                  T* __restrict__ grad_gamma)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.nbox;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t q[3];
        box_coords(d, i, q);
        T sx, sw;
        neighbourhood_sum(d, t, q, sx, sw);
        grad_gamma[i] = sx;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void adam_kernel(int64_t n, T* __restrict__ x, const T* __restrict__ g,
                                                        T* __restrict__ m1, T* __restrict__ m2, T lr, T beta1,
                                                        T beta2, T eps, T bc1, T bc2, T lo, T hi)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T gi = g[i];
        const T a = beta1 * m1[i] + ((T)1 - beta1) * gi;
        const T v = beta2 * m2[i] + ((T)1 - beta2) * gi * gi;
        m1[i] = a;
        m2[i] = v;
        T xi = x[i] - lr * (a / bc1) / (sqrt(v / bc2) + eps);
        xi = xi < lo ? lo : (xi > hi ? hi : xi);
        x[i] = xi;
    }
}

unsigned blocks_for(int64_t n)
{
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < 1 ? 1 : (b > (1 << 20) ? (1 << 20) : b));
}

}  // namespace

hipError_t launch_design_map(int dtype, const DesignArgs& d, const void* gamma, void* m, void* b, void* gbar,
                             hipStream_t s)
{
    if (d.nbox == 0) return hipSuccess;
    if (dtype == 1)
        hipLaunchKernelGGL(design_map_kernel<double>, dim3(blocks_for(d.nbox)), dim3(kThreads), 0, s, d,
                           (const double*)gamma, (double*)m, (double*)b, (double*)gbar);
    else
        hipLaunchKernelGGL(design_map_kernel<float>, dim3(blocks_for(d.nbox)), dim3(kThreads), 0, s, d,
                           (const float*)gamma, (float*)m, (float*)b, (float*)gbar);
    return hipGetLastError();
}

hipError_t launch_design_adjoint(int dtype, const DesignArgs& d, const void* gamma, const void* grad_m,
                                 const void* grad_b, void* tmp, void* grad_gamma, hipStream_t s)
{
    if (d.nbox == 0) return hipSuccess;
    const dim3 grid(blocks_for(d.nbox));
    if (dtype == 1) {
        hipLaunchKernelGGL(design_adjoint_cells<double>, grid, dim3(kThreads), 0, s, d, (const double*)gamma,
                           (const double*)grad_m, (const double*)grad_b, (double*)tmp);
        hipLaunchKernelGGL(design_adjoint_filter<double>, grid, dim3(kThreads), 0, s, d, (const double*)tmp,
                           (double*)grad_gamma);
    } else {
        hipLaunchKernelGGL(design_adjoint_cells<float>, grid, dim3(kThreads), 0, s, d, (const float*)gamma,
                           (const float*)grad_m, (const float*)grad_b, (float*)tmp);
        hipLaunchKernelGGL(design_adjoint_filter<float>, grid, dim3(kThreads), 0, s, d, (const float*)tmp,
                           (float*)grad_gamma);
    }
    return hipGetLastError();
}

hipError_t launch_adam(int dtype, int64_t n, void* x, const void* g, void* m1, void* m2, double lr, double beta1,
                       double beta2, double eps, double bc1, double bc2, double lo, double hi, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (dtype == 1)
        hipLaunchKernelGGL(adam_kernel<double>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, (double*)x,
                           (const double*)g, (double*)m1, (double*)m2, lr, beta1, beta2, eps, bc1, bc2, lo, hi);
    else
        hipLaunchKernelGGL(adam_kernel<float>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, (float*)x,
                           (const float*)g, (float*)m1, (float*)m2, (float)lr, (float)beta1, (float)beta2,
                           (float)eps, (float)bc1, (float)bc2, (float)lo, (float)hi);
    return hipGetLastError();
}

}  // namespace fdw
