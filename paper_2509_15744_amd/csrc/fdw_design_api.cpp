// fdwave design chain around the sweeps (Sec. 2.3): the material map of a design field
// (filter, projection, clip, affine map), its chain rule and the Adam update.

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "fdw_aux.h"
#include "fdw_host.h"

using namespace fdh;

namespace {

// Design description -> kernel arguments, with the checks the header lists.  2D grids
// map to the internal three-axis form with a unit middle axis.
int design_args(const fd_design* D, fdw::DesignArgs* d)
{
    if (!D) return fail(FD_E_ARG, "design is null");
    if (D->ndim != 2 && D->ndim != 3) return fail(FD_E_ARG, "design ndim must be 2 or 3");
    if (D->dtype != FD_F32 && D->dtype != FD_F64) return fail(FD_E_ARG, "design dtype must be FD_F32 or FD_F64");
    const int map[3] = {0, D->ndim == 3 ? 1 : -1, D->ndim == 3 ? 2 : 1};
    d->nbox = 1;
    for (int ax = 0; ax < 3; ++ax) {
        const int src = map[ax];
        const int64_t n = src < 0 ? 1 : D->shape[src];
        const int64_t o = src < 0 ? 0 : D->origin[src];
        const int64_t e = src < 0 ? 1 : D->extent[src];
        if (n < 1 || n > (1 << 30)) return fail(FD_E_ARG, "design grid extent out of range");
        if (e < 1 || o < 0 || o + e > n) return fail(FD_E_ARG, "design box must lie inside the grid");
        d->n[ax] = n;
        d->o[ax] = o;
        d->e[ax] = e;
        d->nbox *= e;
    }
    const double rf = D->filter_radius;
    if (!std::isfinite(rf) || rf > 32.0) return fail(FD_E_ARG, "filter_radius must be finite and at most 32");
    d->rf = rf > 1.0 ? rf : 1.0;
    d->R = (int)std::ceil(d->rf) - 1;
    if (!std::isfinite(D->beta)) return fail(FD_E_ARG, "beta must be finite");
    d->proj = D->beta > 0.0;
    d->beta = D->beta;
    d->eta = D->eta;
    if (d->proj) {
        if (!(D->eta >= 0.0 && D->eta <= 1.0)) return fail(FD_E_ARG, "eta must lie in [0, 1]");
        d->th0 = std::tanh(D->beta * D->eta);
        d->hnorm = d->th0 + std::tanh(D->beta * (1.0 - D->eta));
    } else {
        d->th0 = 0.0;
        d->hnorm = 1.0;
    }
    if (!(D->lo <= D->hi) || std::isnan(D->lo) || std::isnan(D->hi))
        return fail(FD_E_ARG, "clip interval needs lo <= hi");
    d->lo = D->lo;
    d->hi = D->hi;
    for (double v : {D->m0, D->dm, D->b0, D->db})
        if (!std::isfinite(v)) return fail(FD_E_ARG, "material map coefficients must be finite");
    d->m0 = D->m0;
    d->dm = D->dm;
    d->b0 = D->b0;
    d->db = D->db;
    return FD_OK;
}

int design_fields(const fd_design* D, const fdw::DesignArgs& d, const void* box_field, const char* box_name,
                  const void* g1, const char* n1, const void* g2, const char* n2)
{
    const size_t es = dsize(D->dtype);
    const size_t gb = (size_t)(d.n[0] * d.n[1] * d.n[2]) * es;
    int rc = check_dev(box_field, (size_t)d.nbox * es, box_name);
    if (rc) return rc;
    if ((rc = check_dev(g1, gb, n1))) return rc;
    return check_dev(g2, gb, n2);
}

}  // namespace

extern "C" {

int fd_design_map(const fd_design* design, const void* gamma, void* m, void* b, void* gamma_bar, void* stream)
{
    g_err.clear();
    fdw::DesignArgs d;
    int rc = design_args(design, &d);
    if (rc) return rc;
    if ((rc = design_fields(design, d, gamma, "gamma", m, "m", b, "b"))) return rc;
    if (gamma_bar && (rc = check_dev(gamma_bar, (size_t)d.nbox * dsize(design->dtype), "gamma_bar"))) return rc;
    HIPCHK(fdw::launch_design_map(design->dtype, d, gamma, m, b, gamma_bar, (hipStream_t)stream));
    return FD_OK;
}

int fd_design_adjoint(const fd_design* design, const void* gamma, const void* grad_m, const void* grad_b,
                      void* grad_gamma, void* stream)
{
    g_err.clear();
    fdw::DesignArgs d;
    int rc = design_args(design, &d);
    if (rc) return rc;
    if ((rc = design_fields(design, d, gamma, "gamma", grad_m, "grad_m", grad_b, "grad_b"))) return rc;
    const size_t bb = (size_t)d.nbox * dsize(design->dtype);
    if ((rc = check_dev(grad_gamma, bb, "grad_gamma"))) return rc;
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    void* tmp = nullptr;
    HIPCHK(sc.get(&tmp, bb));
    HIPCHK(fdw::launch_design_adjoint(design->dtype, d, gamma, grad_m, grad_b, tmp, grad_gamma, s));
    return FD_OK;
}

int fd_adam_step(int64_t n, int32_t dtype, void* x, const void* grad, void* m1, void* m2, int32_t step,
                 double lr, double beta1, double beta2, double eps, double lo, double hi, void* stream)
{
    g_err.clear();
    if (n < 0) return fail(FD_E_ARG, "n is negative");
    if (dtype != FD_F32 && dtype != FD_F64) return fail(FD_E_ARG, "dtype must be FD_F32 or FD_F64");
    if (step < 1) return fail(FD_E_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(FD_E_ARG, "beta1 and beta2 must lie in [0, 1)");
    if (!(eps >= 0.0) || !std::isfinite(eps) || !std::isfinite(lr))
        return fail(FD_E_ARG, "eps and lr must be finite, eps >= 0");
    if (!(lo <= hi)) return fail(FD_E_ARG, "clip interval needs lo <= hi");
    const size_t bytes = (size_t)n * dsize(dtype);
    int rc;
    if ((rc = check_dev(x, bytes, "x")) || (rc = check_dev(grad, bytes, "grad")) ||
        (rc = check_dev(m1, bytes, "m1")) || (rc = check_dev(m2, bytes, "m2")))
        return rc;
    const double bc1 = 1.0 - std::pow(beta1, step);   // > 0 for beta1 in [0, 1)
    const double bc2 = 1.0 - std::pow(beta2, step);
    HIPCHK(fdw::launch_adam(dtype, n, x, grad, m1, m2, lr, beta1, beta2, eps, bc1, bc2, lo, hi, (hipStream_t)stream));
    return FD_OK;
}

}  // extern "C"
