// fdwave C-ABI entry points for single problems: the forward solve, the misfit, the
// memory-efficient sensitivity of the paper's Algorithm 1 (fused and as two halves),
// the exact re-simulation gradient, the variable-material scheme and the propagation
// test hook.  The shared host runtime is fdw_host.cpp, the kernels live in the .hip
// files.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fdw_aux.h"
#include "fdw_host.h"

using namespace fdh;

namespace {

// Working arrays the fused call makes once for both halves: c in the sweep's row
// layout and the partial sums of the kernel terms (null members: the half makes its own).
struct Shared {
    const void* cp = nullptr;
    void* part = nullptr;
    PairPlan pp;
    PairSweep pw;
    bool made = false;
};

// The two-step launch plan of a half (or the fused call's), when its sweeps use them.
int pair_setup(const Geo& G, const fd_acq* acq, hipStream_t s, Scratch& sc, PairPlan* pp, PairSweep* pw)
{
    if (!use_pairs(G, acq)) return FD_OK;
    return make_pair_sweep(G, acq, s, sc, pp, pw);
}

// `own_state`: the state arrays were allocated by the library itself in this call.
// `ext`: take scratch from this (arena) instead of the stream-ordered pool.
int sens_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
                 const void* observed, const fd_state* st, void* traces, double* J_host,
                 const fd_opts* opts, hipStream_t s, bool own_state, Scratch* ext = nullptr,
                 const Shared* sh = nullptr)
{
    Scratch local(s);
    Scratch& sc = ext ? *ext : local;
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, true);
    if (rc) return rc;
    if (!own_state && (rc = check_state(st, G, nt, acq))) return rc;
    const size_t tb = (size_t)nt * acq->nrec * dsize(G.dtype);
    if ((rc = check_dev(observed, tb, "observed"))) return rc;
    if (traces && (rc = check_dev(traces, tb, "traces"))) return rc;
    pad_rows(&G);
    const void* cp = sh && sh->made ? sh->cp : nullptr;
    if (!(sh && sh->made) && (rc = padded_field(G, c, sc, s, &cp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    const int ns = nshots(acq);
    VdWork w;
    if ((rc = vd_work(G, st, nullptr, ns, own_state, false, sc, s, &w))) return rc;
    void* part = sh && sh->made ? sh->part : nullptr;
    if (!(sh && sh->made) && (rc = partial_buffer(G, sc, &part))) return rc;
    PairPlan pp_own;
    PairSweep pw_own;
    if (!(sh && sh->made) && (rc = pair_setup(G, acq, s, sc, &pp_own, &pw_own))) return rc;
    const PairSweep* pw = sh && sh->made ? &sh->pw : &pw_own;
    if ((rc = forward_sweep(G, P, cp, acq, dt, nt, observed, w.st.u_a, w.st.u_b, w.st.acc, st->residual,
                            traces, s, VdFields(), part, pw)))
        return rc;
    if ((rc = work_out(G, w, st, nullptr, ns, s))) return rc;   // back to the caller's dense layout
    if (J_host) {
        double ss = 0.0;
        if ((rc = misfit_sum(G.dtype, st->residual, nullptr, nullptr, (int64_t)nt * acq->nrec, s, sc, &ss)))
            return rc;
        *J_host = 0.5 * dt * ss;
        if (!std::isfinite(*J_host)) return fail(FD_E_NONFINITE, "misfit is not finite");
    }
    return FD_OK;
}

int sens_backward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt, double k,
                  const fd_state* st, double grad_scale, void* grad, const fd_opts* opts, hipStream_t s,
                  bool own_state, Scratch* ext = nullptr, const Shared* sh = nullptr)
{
    Scratch local(s);
    Scratch& sc = ext ? *ext : local;
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, false);
    if (rc) return rc;
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    if (!std::isfinite(grad_scale)) return fail(FD_E_ARG, "grad_scale must be finite");
    if (!own_state && (rc = check_state(st, G, nt, acq))) return rc;
    if ((rc = check_dev(grad, G.ncell * dsize(G.dtype), "grad_c"))) return rc;
    pad_rows(&G);
    const void* cp = sh && sh->made ? sh->cp : nullptr;
    if (!(sh && sh->made) && (rc = padded_field(G, c, sc, s, &cp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, true, s, sc, &P))) return rc;
    VdWork w;
    if ((rc = vd_work(G, st, nullptr, nshots(acq), own_state, true, sc, s, &w))) return rc;
    void* part = sh && sh->made ? sh->part : nullptr;
    if (!(sh && sh->made) && (rc = partial_buffer(G, sc, &part))) return rc;
    PairPlan pp_own;
    PairSweep pw_own;
    if (!(sh && sh->made) && (rc = pair_setup(G, acq, s, sc, &pp_own, &pw_own))) return rc;
    const PairSweep* pw = sh && sh->made ? &sh->pw : &pw_own;
    if ((rc = backward_sweep(G, P, cp, acq, dt, nt, k, w.st.u_a, w.st.u_b, w.st.acc, st->residual, s,
                             VdFields(), part, pw)))
        return rc;
    if (G.pitch == G.n2) {
        HIPCHK(fdw::launch_finalize(G.dtype, G.acc_dtype, G.ncell, w.st.acc, c, grad_scale / k, grad, s));
    } else {   // finalise in the padded layout, then copy the rows out
        const size_t es = dsize(G.dtype);
        void* t = nullptr;
        HIPCHK(sc.get(&t, G.ncell_pad * es));
        HIPCHK(fdw::launch_finalize(G.dtype, G.acc_dtype, G.ncell_pad, w.st.acc, cp, grad_scale / k, t, s));
        if ((rc = copy_rows(grad, G.n2, t, G.pitch, es, (int64_t)G.n0 * G.n1, G.n2, s))) return rc;
    }
    return FD_OK;
}

// Mass and stiffness of the variable-material scheme: finite and positive, and the
// time step inside the sufficient stability bound dt sqrt(d max b / min m) <= dx (the
// Gershgorin bound of the scaled operator with the second-order symbol).
int check_material(const Geo& G, const void* m, const void* b, double dt, hipStream_t s, Scratch& sc)
{
    void* part = nullptr;
    void* out = nullptr;
    HIPCHK(sc.get(&part, sizeof(double) * 3 * fdw::kReduceBlocks));
    HIPCHK(sc.get(&out, sizeof(double) * 7));
    HIPCHK(fdw::launch_speed_stats(G.dtype, m, G.ncell, (double*)out, (double*)part, s));
    HIPCHK(fdw::launch_speed_stats(G.dtype, b, G.ncell, (double*)out + 3, (double*)part, s));
    double h[7];
    HIPCHK(hipMemcpyAsync(h, out, sizeof(double) * 6, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[2] > 0 || h[5] > 0) return fail(FD_E_NONFINITE, "material field has non-finite entries");
    if (!(h[1] > 0.0) || !(h[4] > 0.0)) return fail(FD_E_NONFINITE, "mass and stiffness must be positive");
    // Leapfrog is stable when dt^2 lambda_max < 4 for the largest eigenvalue of
    // M^-1 K; its Gershgorin bound s_max / dx^2 is exact for a homogeneous medium
    // (dt sqrt(d b/m)/dx <= 1) and stays local where materials mix.
    HIPCHK(fdw::launch_vd_bound(G.dtype, m, b, G.n0, G.n1, G.n2, (double*)out + 6, (double*)part, s));
    HIPCHK(hipMemcpyAsync(h + 6, (double*)out + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double courant = 0.5 * dt * std::sqrt(h[6]) / G.dx;
    if (!(courant <= 1.0 + 1e-12)) {
        char buf[200];
        snprintf(buf, sizeof buf, "dt sqrt(max Gershgorin row sum of M^-1 K) / 2 = %.6g exceeds 1", courant);
        return fail(FD_E_CFL, buf);
    }
    return FD_OK;
}

// Grid, options and launch shape of the variable-material scheme: second order only,
// tile variants 1 and 2, one wavefield per launch.
int vd_setup(const fd_grid* grid, const fd_opts* opts, Geo* G)
{
    int rc = check_grid(grid, opts, G);
    if (rc) return rc;
    if (grid->order != 2) return fail(FD_E_ARG, "the variable-material scheme is second order (order 2)");
    if (G->auto_variant) {
        // 3D: 64 x 4 tiles with two cells per lane (256-thread blocks) measured fastest
        // on 1024^3 (132.6 against 119.6 Gcell-updates/s for 64 x 8 tiles with one cell
        // per lane and 125.9 with two rows per thread); one cell per lane fits every
        // extent.  2D: one cell per lane.
        G->variant = (G->ndim == 3 && G->n2 % 2 == 0) ? 5 : 1;
        G->auto_variant = false;
    } else if (G->variant != 1 && G->variant != 2 && G->variant != 5 && !(G->ndim == 3 && G->variant == 7) &&
               !(G->ndim == 2 && G->variant == 4)) {
        return fail(FD_E_ARG, "the variable-material scheme runs tile variants 1, 2 and 5 (3D also 7, 2D also 4)");
    }
    G->max_group = 1;
    G->variant_plain = 0;   // one launch shape for every launch
    // In 2D a block's march along axis 0 reuses only two neighbour rows from
    // registers while serialising its rows; two-row chunks keep the most blocks in
    // flight and measured fastest (one row ties, longer chunks lose steadily).
    if (G->ndim == 2 && G->chunk == 0) G->chunk = 2;
    pad_rows(G);
    return FD_OK;
}

// Validation shared by the two halves of the variable-material gradient.
int vd_prepare(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt, int nt,
               const fd_opts* opts, Geo* G)
{
    int rc = vd_setup(grid, opts, G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if (!acq) return fail(FD_E_ARG, "acq is null");
    if ((rc = check_acq(acq, *G, nt))) return rc;
    const size_t es = dsize(G->dtype);
    if ((rc = check_dev(m, G->ncell * es, "m"))) return rc;
    if ((rc = check_dev(b, G->ncell * es, "b"))) return rc;
    return FD_OK;
}

int check_vd_state(const fd_state* st, const void* acc_b, const Geo& G, int nt, const fd_acq* acq)
{
    int rc = check_state(st, G, nt, acq);
    if (rc) return rc;
    return check_dev(acc_b, G.ncell * dsize(G.acc_dtype), "acc_b");
}

// First half: forward sweep with cost, adjoint force and both kernel terms of u.
int vd_sens_forward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt, int nt,
                    const void* observed, const fd_state* st, void* acc_b, void* traces, double* J_host,
                    const fd_opts* opts, hipStream_t s, bool own_state)
{
    Geo G;
    int rc = vd_prepare(grid, m, b, acq, dt, nt, opts, &G);
    if (rc) return rc;
    if (!own_state && (rc = check_vd_state(st, acc_b, G, nt, acq))) return rc;
    const size_t tb = (size_t)nt * acq->nrec * dsize(G.dtype);
    if ((rc = check_dev(observed, tb, "observed"))) return rc;
    if (traces && (rc = check_dev(traces, tb, "traces"))) return rc;
    Scratch sc(s);
    if ((rc = check_material(G, m, b, dt, s, sc))) return rc;
    const void *mp = nullptr, *bp = nullptr;
    if ((rc = padded_material(G, m, b, sc, s, &mp, &bp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    const int ns = nshots(acq);
    VdWork w;
    if ((rc = vd_work(G, st, acc_b, ns, own_state, false, sc, s, &w))) return rc;
    VdFields vd;
    vd.stiff = bp;
    vd.acc_b = w.acc_b;
    void* part = nullptr;
    if ((rc = partial_buffer(G, sc, &part)) || (rc = partial_buffer(G, sc, &vd.part_b))) return rc;
    if ((rc = forward_sweep(G, P, mp, acq, dt, nt, observed, w.st.u_a, w.st.u_b, w.st.acc, st->residual, traces,
                            s, vd, part)))
        return rc;
    if ((rc = work_out(G, w, st, acc_b, ns, s))) return rc;   // back to the caller's dense layout
    if (J_host) {
        double ss = 0.0;
        if ((rc = misfit_sum(G.dtype, st->residual, nullptr, nullptr, (int64_t)nt * acq->nrec, s, sc, &ss)))
            return rc;
        *J_host = 0.5 * dt * ss;
        if (!std::isfinite(*J_host)) return fail(FD_E_NONFINITE, "misfit is not finite");
    }
    return FD_OK;
}

// Second half: superposed backward sweep from the state (consumed) and
//   grad_m = s (K_m(u,u) - K_m(v,v)) / (2k),  grad_b = -s (dt^2/dx^2)(K_b(u,u) - K_b(v,v)) / (2k)
// with s = grad_scale.
int vd_sens_backward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt, int nt,
                     double k, const fd_state* st, void* acc_b, double grad_scale, void* grad_m, void* grad_b,
                     const fd_opts* opts, hipStream_t s, bool own_state)
{
    Geo G;
    int rc = vd_prepare(grid, m, b, acq, dt, nt, opts, &G);
    if (rc) return rc;
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    if (!std::isfinite(grad_scale)) return fail(FD_E_ARG, "grad_scale must be finite");
    if (!own_state && (rc = check_vd_state(st, acc_b, G, nt, acq))) return rc;
    const size_t es = dsize(G.dtype);
    if ((rc = check_dev(grad_m, G.ncell * es, "grad_m"))) return rc;
    if ((rc = check_dev(grad_b, G.ncell * es, "grad_b"))) return rc;
    Scratch sc(s);
    const void *mp = nullptr, *bp = nullptr;
    if ((rc = padded_material(G, m, b, sc, s, &mp, &bp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, true, s, sc, &P))) return rc;
    VdWork w;
    if ((rc = vd_work(G, st, acc_b, nshots(acq), own_state, true, sc, s, &w))) return rc;
    VdFields vd;
    vd.stiff = bp;
    vd.acc_b = w.acc_b;
    void* part = nullptr;
    if ((rc = partial_buffer(G, sc, &part)) || (rc = partial_buffer(G, sc, &vd.part_b))) return rc;
    if ((rc = backward_sweep(G, P, mp, acq, dt, nt, k, w.st.u_a, w.st.u_b, w.st.acc, st->residual, s, vd, part)))
        return rc;
    const double sm = grad_scale * 0.5 / k;
    const double sb = -grad_scale * dt * dt / (G.dx * G.dx) * 0.5 / k;
    if (G.pitch == G.n2) {
        HIPCHK(fdw::launch_scale(G.dtype, G.acc_dtype, G.ncell, w.st.acc, sm, grad_m, s));
        HIPCHK(fdw::launch_scale(G.dtype, G.acc_dtype, G.ncell, w.acc_b, sb, grad_b, s));
    } else {   // scale in the padded layout, then copy the rows out
        void *tm = nullptr, *tbuf = nullptr;
        HIPCHK(sc.get(&tm, G.ncell_pad * es));
        HIPCHK(sc.get(&tbuf, G.ncell_pad * es));
        HIPCHK(fdw::launch_scale(G.dtype, G.acc_dtype, G.ncell_pad, w.st.acc, sm, tm, s));
        HIPCHK(fdw::launch_scale(G.dtype, G.acc_dtype, G.ncell_pad, w.acc_b, sb, tbuf, s));
        const int64_t rows = (int64_t)G.n0 * G.n1;
        if ((rc = copy_rows(grad_m, G.n2, tm, G.pitch, es, rows, G.n2, s))) return rc;
        if ((rc = copy_rows(grad_b, G.n2, tbuf, G.pitch, es, rows, G.n2, s))) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    return FD_OK;
}

int vd_gradient(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt, int nt,
                const void* observed, double k, void* grad_m, void* grad_b, double* J_host, void* traces,
                const fd_opts* opts, hipStream_t s)
{
    Geo G;
    int rc = vd_prepare(grid, m, b, acq, dt, nt, opts, &G);
    if (rc) return rc;
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    Scratch sc(s);
    const size_t es = dsize(G.dtype);
    const int ns = nshots(acq);
    fd_state st;
    void* accb = nullptr;
    HIPCHK(sc.get(&st.u_a, G.ncell_pad * es * ns));
    HIPCHK(sc.get(&st.u_b, G.ncell_pad * es * ns));
    HIPCHK(sc.get(&st.acc, G.ncell_pad * dsize(G.acc_dtype)));
    HIPCHK(sc.get(&accb, G.ncell_pad * dsize(G.acc_dtype)));
    HIPCHK(sc.get(&st.residual, std::max<size_t>((size_t)nt * acq->nrec * es, es)));
    if ((rc = vd_sens_forward(grid, m, b, acq, dt, nt, observed, &st, accb, traces, J_host, opts, s, true)))
        return rc;
    return vd_sens_backward(grid, m, b, acq, dt, nt, k, &st, accb, 1.0, grad_m, grad_b, opts, s, true);
}

int vd_forward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt, int nt,
               void* traces, const fd_opts* opts, hipStream_t s)
{
    Geo G;
    int rc = vd_setup(grid, opts, &G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if (!acq) return fail(FD_E_ARG, "acq is null");
    if ((rc = check_acq(acq, G, nt))) return rc;
    const size_t es = dsize(G.dtype);
    if ((rc = check_dev(m, G.ncell * es, "m"))) return rc;
    if ((rc = check_dev(b, G.ncell * es, "b"))) return rc;
    if ((rc = check_dev(traces, (size_t)nt * acq->nrec * es, "traces"))) return rc;
    Scratch sc(s);
    if ((rc = check_material(G, m, b, dt, s, sc))) return rc;
    const void *mp = nullptr, *bp = nullptr;
    if ((rc = padded_material(G, m, b, sc, s, &mp, &bp))) return rc;
    const int ns = nshots(acq);
    void *ua = nullptr, *ub = nullptr;
    HIPCHK(sc.get(&ua, G.ncell_pad * es * ns));
    HIPCHK(sc.get(&ub, G.ncell_pad * es * ns));
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    VdFields vd;
    vd.stiff = bp;
    if ((rc = forward_sweep(G, P, mp, acq, dt, nt, nullptr, ua, ub, nullptr, nullptr, traces, s, vd)))
        return rc;
    HIPCHK(hipStreamSynchronize(s));
    return FD_OK;
}

// Launch shape of the re-simulation backward sweep: a variant that carries two fields
// per launch (the remembered choice for two shots, else for one shot, when it can).
int pair_variant(Geo& G)
{
    if (G.auto_variant) {
        if (!apply_tuned(G, 2)) apply_tuned(G, 1);
        G.auto_variant = false;
        if (fdw::variant_shape(G.ndim, G.variant).max_shots < 2) {
            // one cell per lane, 64-plane chunks: on 1024^3 the re-simulation ran at
            // 159.8 Gcell-updates/s, against 145.3 with two cells per lane and the
            // library's chunk (140.3 and 134.2 with two cells per lane and 64- or
            // 1024-plane chunks)
            G.variant = 1;
            G.chunk = 64;
        }
    }
    if (fdw::variant_shape(G.ndim, G.variant).max_shots < 2)
        return fail(FD_E_ARG, "variant " + std::to_string(G.variant) + " cannot carry two fields per launch");
    G.max_group = 0;
    return FD_OK;
}

// Exact discrete gradient without stored history (re-simulation): after a forward sweep
// without kernel accumulation, u is stepped backward from (u^nt, u^{nt-1}) by the same
// scheme (time-reversible) together with the adjoint field mu, whose sweep starts from
// mu^nt = 0, mu^{nt-1} = coef fdag^nt (the exact discrete adjoint that the superposition
// of Sec. 4 approximates, with the kernel of Eq. kernel2 in its discrete form), and the
// launch accumulates the cross kernel sum_n (u^{n+1} - u^n)(mu^{n+1} - mu^n); then
// grad_c = 2 acc / c^3.  Shot s keeps u at slot s and mu at slot nshot + s of the two
// field buffers.
int exact_gradient(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
                   const void* observed, void* grad, double* J_host, void* traces,
                   const fd_opts* opts, hipStream_t s)
{
    Scratch sc(s);
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, true);
    if (rc) return rc;
    const size_t es = dsize(G.dtype);
    const size_t tb = (size_t)nt * acq->nrec * es;
    if ((rc = check_dev(observed, tb, "observed"))) return rc;
    if (traces && (rc = check_dev(traces, tb, "traces"))) return rc;
    if ((rc = check_dev(grad, G.ncell * es, "grad_c"))) return rc;
    const int ns = nshots(acq);
    const size_t half = G.ncell * es * ns;
    void *ua = nullptr, *ub = nullptr, *acc = nullptr, *resid = nullptr;
    HIPCHK(sc.get(&ua, 2 * half));
    HIPCHK(sc.get(&ub, 2 * half));
    HIPCHK(sc.get(&acc, G.ncell * dsize(G.acc_dtype)));
    HIPCHK(sc.get(&resid, std::max<size_t>(tb, es)));

    Geo Gf = G;
    Plan Pf;
    if ((rc = make_plan(Gf, acq, false, s, sc, &Pf))) return rc;
    if ((rc = forward_sweep(Gf, Pf, c, acq, dt, nt, observed, ua, ub, nullptr, resid, traces, s)))
        return rc;
    if (J_host) {
        double ss = 0.0;
        if ((rc = misfit_sum(G.dtype, resid, nullptr, nullptr, (int64_t)nt * acq->nrec, s, sc, &ss)))
            return rc;
        *J_host = 0.5 * dt * ss;
        if (!std::isfinite(*J_host)) return fail(FD_E_NONFINITE, "misfit is not finite");
    }

    Geo Gb = G;
    if ((rc = pair_variant(Gb))) return rc;
    Plan Pb;
    if ((rc = make_plan(Gb, acq, true, s, sc, &Pb, true))) return rc;
    void* up = nullptr;   // u^{nt-1}
    void* ul = nullptr;   // u^nt
    final_levels(ua, ub, nt, &up, &ul);
    HIPCHK(hipMemsetAsync((char*)up + half, 0, half, s));
    HIPCHK(hipMemsetAsync((char*)ul + half, 0, half, s));
    HIPCHK(hipMemsetAsync(acc, 0, G.ncell * dsize(G.acc_dtype), s));
    const double rec_scale = -1.0 / dt;   // fdag^n = -residual^n / dt
    if (acq->nrec > 0)
        HIPCHK(fdw::launch_terminal_exact(G.dtype, G.acc_dtype, Pb.nuniq, Pb.d_ucell, Pb.d_uoff, Pb.d_uidx,
                                          Pb.d_ushot, 0, ns, G.ncell, (int64_t)G.ncell * ns, c, dt * dt,
                                          ul, up, acc, (const char*)resid + (size_t)(nt - 1) * acq->nrec * es,
                                          rec_scale, s));
    fdw::StepArgs a = base_args(Gb, Pb, c, dt);
    a.shot_stride = (int64_t)G.ncell_pad * ns;   // slot 1 (mu) of shot s sits nshot fields after its u
    a.acc = acc;
    if ((rc = partial_buffer(G, sc, &a.part))) return rc;
    a.acc_cross = 1;
    a.wavelet = acq->wavelet;
    a.nsrc = acq->nsrc;
    a.inject_rec = 1;
    a.resid = resid;
    a.nrec = acq->nrec;
    a.rec_scale = rec_scale;
    SweepTimer tm(G.timing != nullptr && nt > 1, s);
    tm.start();
    for (int gi = 0; gi < (int)Pb.groups.size(); ++gi) {
        const Group& gr = Pb.groups[gi];
        char* xj = (char*)up + (size_t)gr.g0 * G.ncell * es;   // level j
        char* xn = (char*)ul + (size_t)gr.g0 * G.ncell * es;   // level j+1, overwritten by j-1
        for (int j = nt - 1; j >= 1; --j) {
            a.ucur = xj;
            a.unew = xn;
            a.row_src = j;
            a.row_rec = j - 1;
            set_acc_at(a, nt - 1 - j, nt - 1, 1);   // intervals nt-2..0
            if ((rc = step(Gb, Pb, gi, a, s))) return rc;
            std::swap(xj, xn);
        }
    }
    tm.stop();
    if (G.timing) {
        G.timing->bwd_ms = tm.ms();
        G.timing->bwd_launches = (nt - 1) * (int)Pb.groups.size();
    }
    HIPCHK(fdw::launch_finalize(G.dtype, G.acc_dtype, G.ncell, acc, c, -2.0, grad, s));
    HIPCHK(hipStreamSynchronize(s));
    return FD_OK;
}


// Upper bound of the device scratch of one gradient call on grid G (checked, rows not yet
// padded): `total` as the stream-ordered pool sees it (counting no reuse of freed pieces), and
// `arena` when every piece is a new one (the no-allocation entry point).
struct WorkBytes {
    size_t total = 0, arena = 0;
};

WorkBytes workspace_bytes(Geo G, const fd_acq* acq, int nt, int nshots)
{
    const size_t es = dsize(G.dtype);
    const size_t ns = nshots > 1 ? (size_t)nshots : 1;
    const size_t nsrc = acq && acq->nsrc > 0 ? (size_t)acq->nsrc : 0;
    const size_t nrec = acq && acq->nrec > 0 ? (size_t)acq->nrec : 0;
    pad_rows(&G);   // the call's own arrays use the padded row layout
    const size_t np = (size_t)G.ncell_pad;
    const bool padded = G.pitch != G.n2;
    size_t bytes = 2 * ns * np * es + np * 8 + (size_t)nt * nrec * es;
    if (G.dtype == FD_F32) bytes += np * sizeof(float);   // partial sums of the kernel terms
    if (padded) bytes += 2 * np * es;   // padded copy of c, finalisation rows
    // the largest block count of any tile variant with one plane per block
    int64_t per_plane = 1;
    for (int v = 1; v <= fdw::variant_count(G.ndim); ++v) {
        const fdw::Variant w = fdw::variant_shape(G.ndim, v);
        per_plane = std::max<int64_t>(per_plane, (int64_t)((G.n2 + w.tz - 1) / w.tz) * ((G.n1 + w.ty - 1) / w.ty));
    }
    const size_t nblk = (size_t)(per_plane * G.n0);
    const size_t events = nsrc + nrec;
    // each shot group of a plan has its own block offsets (at most one group per shot)
    const size_t plan = ns * ((nblk + 1) * sizeof(int32_t) + 256) +
                        events * (sizeof(fdw::Event) + sizeof(fdw::EvPlane)) +
                        nrec * (sizeof(int64_t) + 3 * sizeof(int32_t)) + sizeof(int32_t) + 4096;
    WorkBytes w;
    // the launch plans of both halves, each with a second launch shape, and the
    // reduction partials of the speed check and of the misfit, none of them reused
    w.total = bytes + 4 * plan + sizeof(double) * (4 * fdw::kReduceBlocks + 16);
    // and the 256-byte alignment of every piece
    w.arena = w.total + 256 * (8 * ns + 64);
    return w;
}

// Alg. 1 end to end with the library's own state; `ext` as for the halves.
int adjoint_sensitivity(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
                        const void* observed, double k, void* grad_c, double* J_host, void* traces_or_null,
                        const fd_opts* opts, hipStream_t s, Scratch* ext)
{
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if (!acq) return fail(FD_E_ARG, "acq is null");
    if (acq->nrec < 0) return fail(FD_E_ARG, "receiver count is negative");
    if (acq->nshot < 0) return fail(FD_E_ARG, "nshot is negative");
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    Scratch local(s);
    Scratch& sc = ext ? *ext : local;
    pad_rows(&G);   // the halves' own state is in the (possibly padded) row layout
    fd_state st;
    HIPCHK(sc.get(&st.u_a, G.ncell_pad * dsize(G.dtype) * nshots(acq)));
    HIPCHK(sc.get(&st.u_b, G.ncell_pad * dsize(G.dtype) * nshots(acq)));
    HIPCHK(sc.get(&st.acc, G.ncell_pad * dsize(G.acc_dtype)));
    HIPCHK(sc.get(&st.residual, (size_t)nt * acq->nrec * dsize(G.dtype)));
    // c in the row layout of the sweeps and the partial sums, once for both halves
    if ((rc = check_dev(c, G.ncell * dsize(G.dtype), "c"))) return rc;
    Shared sh;
    if ((rc = padded_field(G, c, sc, s, &sh.cp)) || (rc = partial_buffer(G, sc, &sh.part))) return rc;
    // the two-step plan reads the acquisition's cells: check them first
    if ((rc = check_acq(acq, G, nt)) || (rc = pair_setup(G, acq, s, sc, &sh.pp, &sh.pw))) return rc;
    sh.made = true;
    if ((rc = sens_forward(grid, c, acq, dt, nt, observed, &st, traces_or_null, J_host, opts, s, true, &sc, &sh)))
        return rc;
    return sens_backward(grid, c, acq, dt, nt, k, &st, 1.0, grad_c, opts, s, true, &sc, &sh);
}

// ---------------------------------------------------------------------------
// no-allocation form of the gradient: scratch in a fixed device array per GPU
// ---------------------------------------------------------------------------

constexpr size_t kNoAllocBytes = FD_NOALLOC_BYTES;
static_assert(kNoAllocBytes % 256 == 0, "the array keeps 256-byte pieces aligned");

// Every GPU the library runs on holds its own copy of this array from the library's
// load until the process ends.  Host code never names it beyond the one
// hipGetSymbolAddress per device: kernels get the address kept for their device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocDevice {
    void* ptr = nullptr;        // device address of this device's array
    std::mutex call;            // held for a whole call: calls on one device never overlap
};
std::mutex g_noalloc_mu;
std::map<int, std::unique_ptr<NoAllocDevice>> g_noalloc;

// The current device's array (its address looked up once, with that device current).
int noalloc_device(NoAllocDevice** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc.find(dev);
    if (it == g_noalloc.end()) {
        auto d = std::make_unique<NoAllocDevice>();
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FD_E_DEVICE, "no device address for the scratch array");
        d->ptr = p;
        it = g_noalloc.emplace(dev, std::move(d)).first;
    }
    *out = it->second.get();
    return FD_OK;
}

}  // namespace

extern "C" {

const char* fd_last_error(void) { return g_err.c_str(); }

double fd_cfl_limit(int32_t ndim, int32_t order) { return cfl_limit(ndim, order); }

size_t fd_workspace_bytes(const fd_grid* grid, const fd_acq* acq, int32_t nt, int32_t nshots)
{
    g_err.clear();
    Geo G;
    if (check_grid(grid, nullptr, &G)) return 0;
    if (nt < 0) {
        fail(FD_E_ARG, "nt is negative");
        return 0;
    }
    return workspace_bytes(G, acq, nt, nshots).total;
}

int32_t fd_variant_count(int32_t ndim)
{
    return (ndim == 2 || ndim == 3) ? fdw::variant_count(ndim) : 0;
}

int fd_variant_info(int32_t ndim, int32_t variant, int32_t* tile_z, int32_t* tile_y,
                    int32_t* threads, int32_t* cells_per_lane, int32_t* max_fields)
{
    g_err.clear();
    if (ndim != 2 && ndim != 3) return fail(FD_E_ARG, "ndim must be 2 or 3");
    const fdw::Variant v = fdw::variant_shape(ndim, variant);
    if (v.tz == 0) return fail(FD_E_ARG, "variant out of range");
    if (tile_z) *tile_z = v.tz;
    if (tile_y) *tile_y = v.ty;
    if (threads) *threads = v.threads;
    if (cells_per_lane) *cells_per_lane = v.vz;
    if (max_fields) *max_fields = v.max_shots;
    return FD_OK;
}

int fd_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int32_t nt,
               void* traces, const fd_opts* opts, void* stream)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, true);
    if (rc) return rc;
    if ((rc = check_dev(traces, (size_t)nt * acq->nrec * dsize(G.dtype), "traces"))) return rc;
    pad_rows(&G);
    const void* cp = nullptr;
    if ((rc = padded_field(G, c, sc, s, &cp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    void *ua = nullptr, *ub = nullptr;
    HIPCHK(sc.get(&ua, G.ncell_pad * dsize(G.dtype) * nshots(acq)));
    HIPCHK(sc.get(&ub, G.ncell_pad * dsize(G.dtype) * nshots(acq)));
    return forward_sweep(G, P, cp, acq, dt, nt, nullptr, ua, ub, nullptr, nullptr, traces, s);
}

int fd_misfit(int32_t nt, int32_t nrec, int32_t dtype, double dt, const void* traces,
              const void* observed, void* residual_or_null, double* J_host, void* stream)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (dtype != FD_F32 && dtype != FD_F64) return fail(FD_E_ARG, "dtype must be FD_F32 or FD_F64");
    int rc = check_time(dt, nt);
    if (rc) return rc;
    if (nrec < 0) return fail(FD_E_ARG, "nrec is negative");
    if (!J_host) return fail(FD_E_ARG, "J_host is null");
    const size_t tb = (size_t)nt * nrec * dsize(dtype);
    if ((rc = check_dev(traces, tb, "traces"))) return rc;
    if ((rc = check_dev(observed, tb, "observed"))) return rc;
    if (residual_or_null && (rc = check_dev(residual_or_null, tb, "residual"))) return rc;
    Scratch sc(s);
    double ss = 0.0;
    if ((rc = misfit_sum(dtype, traces, observed, residual_or_null, (int64_t)nt * nrec, s, sc, &ss)))
        return rc;
    *J_host = 0.5 * dt * ss;
    if (!std::isfinite(*J_host)) return fail(FD_E_NONFINITE, "misfit is not finite");
    return FD_OK;
}

int fd_sens_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int32_t nt,
                    const void* observed, const fd_state* state, void* traces_or_null,
                    double* J_host, const fd_opts* opts, void* stream)
{
    g_err.clear();
    return sens_forward(grid, c, acq, dt, nt, observed, state, traces_or_null, J_host, opts,
                        (hipStream_t)stream, false);
}

int fd_sens_backward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int32_t nt,
                     double k, const fd_state* state, double grad_scale, void* grad_c,
                     const fd_opts* opts, void* stream)
{
    g_err.clear();
    return sens_backward(grid, c, acq, dt, nt, k, state, grad_scale, grad_c, opts,
                         (hipStream_t)stream, false);
}

int fd_adjoint_sensitivity(const fd_grid* grid, const void* c, const fd_acq* acq, double dt,
                           int32_t nt, const void* observed, double k, void* grad_c,
                           double* J_host, void* traces_or_null, const fd_opts* opts, void* stream)
{
    g_err.clear();
    return adjoint_sensitivity(grid, c, acq, dt, nt, observed, k, grad_c, J_host, traces_or_null, opts,
                               (hipStream_t)stream, nullptr);
}

int fd_adjoint_sensitivity_noalloc(const fd_grid* grid, const void* c, const fd_acq* acq, double dt,
                                   int32_t nt, const void* observed, double k, void* grad_c,
                                   double* J_host, void* traces_or_null, const fd_opts* opts, void* stream)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if (!acq) return fail(FD_E_ARG, "acq is null");
    if (acq->nsrc < 0 || acq->nrec < 0) return fail(FD_E_ARG, "source or receiver count is negative");
    if (acq->nshot < 0) return fail(FD_E_ARG, "nshot is negative");
    const size_t need = workspace_bytes(G, acq, nt, nshots(acq)).arena;
    if (need > kNoAllocBytes) {
        char buf[240];
        snprintf(buf, sizeof buf,
                 "this problem needs up to %zu bytes of scratch; the no-allocation entry point holds at "
                 "most %zu (FD_NOALLOC_BYTES): use fd_adjoint_sensitivity",
                 need, kNoAllocBytes);
        return fail(FD_E_ARG, buf);
    }
    NoAllocDevice* d = nullptr;
    if ((rc = noalloc_device(&d))) return rc;
    std::lock_guard<std::mutex> lk(d->call);
    Scratch arena(s, d->ptr, kNoAllocBytes);
    rc = adjoint_sensitivity(grid, c, acq, dt, nt, observed, k, grad_c, J_host, traces_or_null, opts, s, &arena);
    // the array is free for the next call only once this call's work has finished
    const hipError_t e = hipStreamSynchronize(s);
    if (rc) return rc;
    HIPCHK(e);
    return FD_OK;
}

int fd_adjoint_exact(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int32_t nt,
                     const void* observed, void* grad_c, double* J_host, void* traces_or_null,
                     const fd_opts* opts, void* stream)
{
    g_err.clear();
    if (!acq) return fail(FD_E_ARG, "acq is null");
    return exact_gradient(grid, c, acq, dt, nt, observed, grad_c, J_host, traces_or_null, opts,
                          (hipStream_t)stream);
}

int fd_vd_forward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt,
                  int32_t nt, void* traces, const fd_opts* opts, void* stream)
{
    g_err.clear();
    return vd_forward(grid, m, b, acq, dt, nt, traces, opts, (hipStream_t)stream);
}

int fd_vd_adjoint_sensitivity(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq,
                              double dt, int32_t nt, const void* observed, double k, void* grad_m,
                              void* grad_b, double* J_host, void* traces_or_null, const fd_opts* opts,
                              void* stream)
{
    g_err.clear();
    return vd_gradient(grid, m, b, acq, dt, nt, observed, k, grad_m, grad_b, J_host, traces_or_null, opts,
                       (hipStream_t)stream);
}

int fd_vd_sens_forward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt,
                       int32_t nt, const void* observed, const fd_state* state, void* acc_b,
                       void* traces_or_null, double* J_host, const fd_opts* opts, void* stream)
{
    g_err.clear();
    return vd_sens_forward(grid, m, b, acq, dt, nt, observed, state, acc_b, traces_or_null, J_host, opts,
                           (hipStream_t)stream, false);
}

int fd_vd_sens_backward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt,
                        int32_t nt, double k, const fd_state* state, void* acc_b, double grad_scale,
                        void* grad_m, void* grad_b, const fd_opts* opts, void* stream)
{
    g_err.clear();
    return vd_sens_backward(grid, m, b, acq, dt, nt, k, state, acc_b, grad_scale, grad_m, grad_b, opts,
                            (hipStream_t)stream, false);
}

int fd_propagate(const fd_grid* grid, const void* coef, void* u_prev, void* u_cur, int32_t nsteps,
                 const fd_opts* opts, void* stream)
{
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if (nsteps < 0) return fail(FD_E_ARG, "nsteps is negative");
    const size_t fb = G.ncell * dsize(G.dtype);
    if ((rc = check_dev(coef, fb, "coef"))) return rc;
    if ((rc = check_dev(u_prev, fb, "u_prev"))) return rc;
    if ((rc = check_dev(u_cur, fb, "u_cur"))) return rc;
    if (nsteps == 0) return FD_OK;
    Scratch sc(s);
    Plan P;
    if ((rc = make_plan(G, nullptr, false, s, sc, &P))) return rc;
    fdw::StepArgs a = base_args(G, P, coef, 1.0);
    a.coef_direct = 1;
    void* prev = u_prev;
    void* cur = u_cur;
    for (int n = 0; n < nsteps; ++n) {
        a.ucur = cur;
        a.unew = prev;
        if ((rc = step(G, P, 0, a, s))) return rc;
        std::swap(prev, cur);
    }
    if (nsteps & 1) {   // newest level sits in u_prev: swap the two buffers' contents
        void* t = nullptr;
        HIPCHK(sc.get(&t, fb));
        HIPCHK(hipMemcpyAsync(t, u_prev, fb, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(u_prev, u_cur, fb, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(u_cur, t, fb, hipMemcpyDeviceToDevice, s));
    }
    return FD_OK;
}

}  // extern "C"
