// Launchers of the kernels that sit around the sweeps: the stability bound of the
// variable-material scheme, the design-field chain of gradient-based design (density
// filter, projection, clip, material map, and its adjoint) and the Adam update.
#pragma once

#include "fdw_internal.h"

namespace fdw {

// Largest Gershgorin row sum (times dx^2) of the mass-scaled variable-material
// operator, into d_out[0]; d_part holds kReduceBlocks doubles.  Extents are the
// internal ones (n1 = 1 for 2D grids).
hipError_t launch_vd_bound(int dtype, const void* m, const void* b, int64_t n0, int64_t n1, int64_t n2,
                           double* d_out, double* d_part, hipStream_t s);

// A box of design cells inside the grid and the chain that turns the design field
// gamma (one value per box cell, C order over the box) into material:
//   filtered   gt_i = sum_k w_ik gamma_k / sum_k w_ik   (w = rf - |x_i - x_k| > 0, k in the box)
//   projected  h_i  = (th0 + tanh(beta (gt_i - eta))) / hnorm      (proj = 1; else h = gt)
//   clipped    g_i  = min(max(h_i, lo), hi)
//   material   m = m0 + g dm,  b = b0 + g db   at the grid cell of box cell i.
// Extents and origin in the internal three-axis form (2D: axis 1 has extent 1).
struct DesignArgs {
    int64_t n[3];
    int64_t o[3];
    int64_t e[3];
    int64_t nbox;
    double rf;      // filter radius in cells, >= 1 (1: no filtering)
    int R;          // largest offset per axis, ceil(rf) - 1
    int proj;
    double beta, eta, th0, hnorm;   // th0 = tanh(beta eta), hnorm = th0 + tanh(beta (1 - eta))
    double lo, hi;
    double m0, dm, b0, db;
};

hipError_t launch_design_map(int dtype, const DesignArgs& d, const void* gamma, void* m, void* b, void* gbar,
                             hipStream_t s);
// dC/dgamma from dC/dm and dC/db (grid fields): the chain rule of the map above, the
// filter's transpose applied in a second pass; tmp holds nbox values.
hipError_t launch_design_adjoint(int dtype, const DesignArgs& d, const void* gamma, const void* grad_m,
                                 const void* grad_b, void* tmp, void* grad_gamma, hipStream_t s);
// One Adam update of x from its gradient, moments m1 and m2 updated in place, bias
// corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t, then x clipped to [lo, hi].
hipError_t launch_adam(int dtype, int64_t n, void* x, const void* g, void* m1, void* m2, double lr, double beta1,
                       double beta2, double eps, double bc1, double bc2, double lo, double hi, hipStream_t s);

}  // namespace fdw
