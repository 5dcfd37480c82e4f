// fdwave batches of independent problems of uneven sizes: every time step of all
// problems is one launch over the union of their tiles (or one persistent launch per
// sweep), with the paper's Algorithm 1 run per problem.
//
// A batch plan holds everything that needs the host (validation, speed and CFL
// checks, block decompositions, event tables, step-argument tables, state arrays);
// a run of the plan only issues kernel launches on the caller's stream, so the
// caller may capture it once in a hipGraph and replay it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fdw_batch.h"
#include "fdw_host.h"

using namespace fdh;

struct fd_batch_plan {
    int nprob = 0;
    Geo G0;                          // launch options shared by all problems
    std::vector<Geo> G;
    std::vector<Plan> P;
    std::vector<fd_problem> probs;   // the caller's problems (device pointers kept)
    std::vector<const void*> cp;     // speed in the sweep layout: caller's c or cpad
    std::vector<void*> cpad;         // padded copy of c, refreshed by every run (or null)
    std::vector<void*> gpad;         // padded finalisation rows (or null)
    std::vector<fd_state> st;        // per problem: two wavefields, accumulator, residuals
    std::vector<void*> part;         // per problem: partial sums of the kernel terms (or null)
    int nfw = 0, nbw = 0, total = 0;
    fdw::StepArgs* d_tab = nullptr;  // (nfw + nbw) rows of nprob step arguments
    int32_t* d_bstart = nullptr;     // first block of each problem in a launch
    double* d_part = nullptr;        // reduction partials
    unsigned* d_bar = nullptr;       // persistent launches: error flag, join counters, per-group progress
    int capacity = 0;                // persistent launches: blocks of the grid
    int ncand = 0;                   // persistent launches: group plans (chunks per group)
    int ngroups = 0;                 // persistent launches: groups of all problems, plan 0
    int32_t* d_candk = nullptr;      // persistent launches: chunks per group of each plan
    int32_t* d_gstart = nullptr;     // persistent launches: first group of each problem, per plan
    long long timeout_ticks = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // sweep timing (opts.timing)
    bool timed = false;
    std::vector<void*> owned;        // stream-ordered allocations, freed by destroy
};

namespace {

// Group plans of a persistent plan.  Each chunk keeps the length the per-step launches
// use (short in 2D: every chunk's march starts with its queue fill, whose loads are in
// flight together), and K consecutive chunks of a tile column form a group, the unit a
// block takes per step and the unit of the waits; a group spans at least r planes (its
// chunks' queues then reach only the adjacent groups).  Plan 0 takes the smallest K at
// which the groups fit the grid (`cap` blocks), the next plans the smallest K at which
// they fit 63/64, 62/64, ... of it, down to half.  How many blocks run together is
// known only inside the launch; the kernel then takes the first plan whose groups do
// not outnumber them, so each block holds one group per step instead of some holding
// two (whose blocks the neighbours' waits would then all pace).  Fills *cand_k
// (ascending) and *gstart (nprob + 1 group starts per plan).
int persistent_group_plans(const std::vector<Plan>& P, const std::vector<Geo>& G, int cap,
                           std::vector<int32_t>* cand_k, std::vector<int32_t>* gstart)
{
    int kmin = 1, kmax = 1;
    for (size_t p = 0; p < P.size(); ++p) {
        kmin = std::max(kmin, (G[p].r + P[p].chunk - 1) / P[p].chunk);
        kmax = std::max(kmax, P[p].nch);
    }
    kmin = std::min(kmin, kmax);
    auto groups_at = [&](int K) {
        int64_t n = 0;
        for (const Plan& q : P) n += (int64_t)q.ntz * q.nty * ((q.nch + K - 1) / K);
        return n;
    };
    auto smallest_fitting = [&](int64_t target) {   // groups_at falls as K grows
        if (groups_at(kmax) > target) return kmax;   // even whole columns exceed it
        int lo = kmin, hi = kmax;
        while (lo < hi) {
            const int mid = lo + (hi - lo) / 2;
            if (groups_at(mid) <= target) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    };
    cand_k->clear();
    for (int i = 0; i <= 32; ++i) {
        const int K = smallest_fitting((int64_t)cap - (int64_t)cap * i / 64);
        if (cand_k->empty() || K > cand_k->back()) cand_k->push_back(K);
    }
    if (groups_at(cand_k->front()) > (1 << 28)) return fail(FD_E_ARG, "too many groups for a persistent launch");
    const size_t np = P.size();
    gstart->assign(cand_k->size() * (np + 1), 0);
    for (size_t j = 0; j < cand_k->size(); ++j) {
        const int K = (*cand_k)[j];
        int32_t* gs = gstart->data() + j * (np + 1);
        for (size_t p = 0; p < np; ++p) {
            const Plan& q = P[p];
            gs[p + 1] = gs[p] + q.ntz * q.nty * ((q.nch + K - 1) / K);
        }
    }
    return FD_OK;
}

int plan_create(const fd_problem* probs, int nprob, const fd_opts* opts, hipStream_t s, fd_batch_plan** out)
{
    if (!out) return fail(FD_E_ARG, "plan output pointer is null");
    *out = nullptr;
    if (!probs || nprob < 1) return fail(FD_E_ARG, "need at least one problem");
    Scratch sc(s);
    auto pl = std::make_unique<fd_batch_plan>();
    fd_batch_plan& B = *pl;
    B.nprob = nprob;
    B.G.resize(nprob);
    B.P.resize(nprob);
    B.probs.assign(probs, probs + nprob);
    std::vector<Geo>& G = B.G;
    int rc;
    for (int p = 0; p < nprob; ++p) {
        const fd_problem& q = probs[p];
        const std::string who = "problem " + std::to_string(p) + ": ";
        if ((rc = check_grid(&q.grid, opts, &G[p]))) return fail(rc, who + g_err);
        G[p].auto_variant = false;   // one launch serves every problem: one shape for all
        if (p > 0 && (G[p].ndim != G[0].ndim || G[p].r != G[0].r || G[p].dtype != G[0].dtype))
            return fail(FD_E_ARG, who + "all problems need the same ndim, order and dtype");
        if ((rc = check_time(q.dt, q.nt))) return fail(rc, who + g_err);
        if (q.acq.nshot > 1) return fail(FD_E_ARG, who + "batched problems have one shot each");
        if ((rc = check_acq(&q.acq, G[p], q.nt))) return fail(rc, who + g_err);
        if (!(q.k != 0.0) || !std::isfinite(q.k)) return fail(FD_E_ARG, who + "k must be finite and non-zero");
        const size_t fb = G[p].ncell * dsize(G[p].dtype);
        const size_t tb = (size_t)q.nt * q.acq.nrec * dsize(G[p].dtype);
        if ((rc = check_dev(q.c, fb, "c"))) return fail(rc, who + g_err);
        if ((rc = check_dev(q.grad_c, fb, "grad_c"))) return fail(rc, who + g_err);
        if ((rc = check_dev(q.observed, tb, "observed"))) return fail(rc, who + g_err);
        if (q.traces && (rc = check_dev(q.traces, tb, "traces"))) return fail(rc, who + g_err);
        // the source and receiver tables are host memory of the caller: the plan keeps
        // its own event tables instead
        B.probs[p].acq.src_cell = nullptr;
        B.probs[p].acq.rec_cell = nullptr;
        B.probs[p].acq.src_shot = nullptr;
        B.probs[p].acq.rec_shot = nullptr;
    }
    B.G0 = G[0];
    {
        // the tile shapes the multi-problem kernels are built for
        const int v = G[0].variant;
        const bool ok = v == 1 || v == 2 || (G[0].ndim == 2 && (v == 4 || v == 5));
        if (!ok) return fail(FD_E_ARG, "batched calls run tile variants 1 and 2 (2D also 4 and 5)");
    }
    if (B.G0.persistent) {
        HIPCHK(fdw::persistent_capacity(G[0].ndim, G[0].r, G[0].dtype, G[0].acc_dtype, G[0].variant, &B.capacity));
        if (B.capacity < 8) return fail(FD_E_DEVICE, "persistent launch: the step kernel does not fit the device");
    }
    {
        std::vector<const Geo*> gs;
        std::vector<const void*> cs;
        std::vector<double> dts;
        for (int p = 0; p < nprob; ++p) {
            gs.push_back(&G[p]);
            cs.push_back(probs[p].c);
            dts.push_back(probs[p].dt);
        }
        if ((rc = check_speeds(gs, cs, dts, s, sc))) return rc;
    }
    // each problem sweeps on rows padded to 64 elements when its extent needs it
    B.cp.resize(nprob);
    B.cpad.assign(nprob, nullptr);
    B.gpad.assign(nprob, nullptr);
    B.st.resize(nprob);
    B.part.assign(nprob, nullptr);
    std::vector<int32_t> bstart(nprob + 1, 0);
    int nt_max = 0;
    for (int p = 0; p < nprob; ++p) {
        pad_rows(&G[p]);
        const size_t es = dsize(G[p].dtype);
        const size_t fb = G[p].ncell_pad * es;
        B.cp[p] = probs[p].c;
        if (G[p].pitch != G[p].n2) {
            HIPCHK(sc.get(&B.cpad[p], fb));
            HIPCHK(sc.get(&B.gpad[p], fb));
            B.cp[p] = B.cpad[p];
        }
        if ((rc = make_plan(G[p], &probs[p].acq, true, s, sc, &B.P[p]))) return rc;
        HIPCHK(sc.get(&B.st[p].u_a, fb));
        HIPCHK(sc.get(&B.st[p].u_b, fb));
        HIPCHK(sc.get(&B.st[p].acc, G[p].ncell_pad * dsize(G[p].acc_dtype)));
        HIPCHK(sc.get(&B.st[p].residual, (size_t)probs[p].nt * probs[p].acq.nrec * es));
        if ((rc = partial_buffer(G[p], sc, &B.part[p]))) return rc;
        bstart[p + 1] = bstart[p] + B.P[p].nblk;
        nt_max = std::max(nt_max, probs[p].nt);
    }
    B.total = bstart[nprob];
    std::vector<int32_t> cand_k, gstart;
    if (B.G0.persistent) {
        if ((rc = persistent_group_plans(B.P, G, B.capacity, &cand_k, &gstart))) return rc;
        B.ncand = (int)cand_k.size();
        B.ngroups = gstart[nprob];
    }
    // step argument tables: forward steps n = 0..nt_max-1, backward steps aligned at
    // their ends (backward step i runs j = nt_p - 1 - i of problem p while j >= 1)
    B.nfw = nt_max;
    B.nbw = nt_max - 1;
    std::vector<fdw::StepArgs> tab((size_t)(B.nfw + std::max(B.nbw, 0)) * nprob);
    for (int p = 0; p < nprob; ++p) {
        const fd_problem& q = probs[p];
        const Plan& P = B.P[p];
        void *prev = B.st[p].u_a, *cur = B.st[p].u_b;
        for (int n = 0; n < B.nfw; ++n) {
            fdw::StepArgs a = base_args(G[p], P, B.cp[p], q.dt);
            a.blk_off = P.groups[0].d_off;
            a.grp = P.groups[0].d_grp;
            a.ev = P.groups[0].d_ev;
            a.active = n < q.nt;
            a.acc = B.st[p].acc;
            a.part = B.part[p];
            set_acc_at(a, n, q.nt - 1, 1);
            a.wavelet = q.acq.wavelet;
            a.nsrc = q.acq.nsrc;
            a.sample = 1;
            a.traces = q.traces;
            a.resid = B.st[p].residual;
            a.obs = q.observed;
            a.nrec = q.acq.nrec;
            a.row_src = a.row_rec = std::min(n, q.nt - 1);
            a.ucur = cur;
            a.unew = prev;
            tab[(size_t)n * nprob + p] = a;
            if (n < q.nt) std::swap(prev, cur);
        }
        void *up = nullptr, *ul = nullptr;
        final_levels(B.st[p].u_a, B.st[p].u_b, q.nt, &up, &ul);
        void *vj = up, *vn = ul;
        for (int i = 0; i < B.nbw; ++i) {
            const int j = q.nt - 1 - i;
            fdw::StepArgs a = base_args(G[p], P, B.cp[p], q.dt);
            a.blk_off = P.groups[0].d_off;
            a.grp = P.groups[0].d_grp;
            a.ev = P.groups[0].d_ev;
            a.active = j >= 1;
            a.acc = B.st[p].acc;
            a.part = B.part[p];
            set_acc_at(a, i, q.nt - 1, -1);
            a.wavelet = q.acq.wavelet;
            a.nsrc = q.acq.nsrc;
            a.inject_rec = 1;
            a.resid = B.st[p].residual;
            a.nrec = q.acq.nrec;
            a.rec_scale = -q.k / q.dt;
            a.row_src = std::max(j, 1);
            a.row_rec = std::max(j - 1, 0);
            a.ucur = vj;
            a.unew = vn;
            tab[(size_t)(B.nfw + i) * nprob + p] = a;
            if (j >= 1) std::swap(vj, vn);
        }
    }
    HIPCHK(sc.get((void**)&B.d_tab, sizeof(fdw::StepArgs) * tab.size()));
    HIPCHK(sc.get((void**)&B.d_bstart, sizeof(int32_t) * bstart.size()));
    HIPCHK(sc.get((void**)&B.d_part, sizeof(double) * fdw::kReduceBlocks));
    HIPCHK(hipMemcpyAsync(B.d_tab, tab.data(), sizeof(fdw::StepArgs) * tab.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.d_bstart, bstart.data(), sizeof(int32_t) * bstart.size(), hipMemcpyHostToDevice, s));
    if (B.G0.persistent) {
        // error flag, join counters and per-group progress, zeroed by kernels in every
        // run; the bounded wait in device wall-clock ticks
        HIPCHK(sc.get((void**)&B.d_bar, sizeof(unsigned) * ((size_t)fdw::kProgressWords + B.ngroups)));
        HIPCHK(sc.get((void**)&B.d_gstart, sizeof(int32_t) * gstart.size()));
        HIPCHK(hipMemcpyAsync(B.d_gstart, gstart.data(), sizeof(int32_t) * gstart.size(), hipMemcpyHostToDevice, s));
        HIPCHK(sc.get((void**)&B.d_candk, sizeof(int32_t) * cand_k.size()));
        HIPCHK(hipMemcpyAsync(B.d_candk, cand_k.data(), sizeof(int32_t) * cand_k.size(), hipMemcpyHostToDevice, s));
        int dev = 0, khz = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const long long us = B.G0.barrier_timeout_us > 0 ? B.G0.barrier_timeout_us : 2000000;
        B.timeout_ticks = std::max(1LL, us * (long long)khz / 1000);
    }
    if (B.G0.timing) {
        B.timed = true;
        for (hipEvent_t& e : B.ev) HIPCHK(hipEventCreate(&e));
    }
    HIPCHK(hipStreamSynchronize(s));   // the host tables die with this frame
    B.owned = sc.release();
    *out = pl.release();
    return FD_OK;
}

// One sweep of the plan: `count` table rows from `first`, per-step launches or one
// persistent launch.
int plan_sweep(const fd_batch_plan& B, int first, int count, hipStream_t s)
{
    const Geo& G0 = B.G0;
    const fdw::StepArgs* rows = B.d_tab + (size_t)first * B.nprob;
    if (G0.persistent) {
        int grid = 0;
        // the join's counters (arrivals, blocks taking part, ranked, per XCD) and the
        // groups' progress start at zero in every sweep (the error flag, word 2, spans
        // the run)
        HIPCHK(fdw::launch_zero(B.d_bar + 4, sizeof(unsigned) * ((size_t)fdw::kProgressWords - 4 + B.ngroups), s));
        const fdw::GroupPlans gp = {B.d_candk, B.d_gstart, B.ncand, B.ngroups};
        HIPCHK(fdw::launch_step_persistent(G0.ndim, G0.r, G0.dtype, G0.acc_dtype, G0.variant, rows, gp, B.nprob,
                                           count, B.d_bar, B.timeout_ticks, s, &grid));
        return FD_OK;
    }
    for (int i = 0; i < count; ++i)
        HIPCHK(fdw::launch_step_multi(G0.ndim, G0.r, G0.dtype, G0.acc_dtype, G0.variant,
                                      rows + (size_t)i * B.nprob, B.d_bstart, B.nprob, B.total, s));
    return FD_OK;
}

// Kernel launches only (no allocation, copy from or to the host, memset or
// synchronisation): a caller may capture a run in a graph and replay it.
int plan_run(fd_batch_plan* B, double* J_dev, hipStream_t s)
{
    if (!B) return fail(FD_E_ARG, "plan is null");
    if (!J_dev) return fail(FD_E_ARG, "J is null");
    const int np = B->nprob;
    int rc;
    for (int p = 0; p < np; ++p) {
        const Geo& G = B->G[p];
        const size_t fb = G.ncell_pad * dsize(G.dtype);
        HIPCHK(fdw::launch_zero(B->st[p].u_a, fb, s));
        HIPCHK(fdw::launch_zero(B->st[p].u_b, fb, s));
        HIPCHK(fdw::launch_zero(B->st[p].acc, G.ncell_pad * dsize(G.acc_dtype), s));
        if (B->cpad[p])   // the caller's c as it is now, in the padded row layout
            HIPCHK(fdw::launch_copy_rows(B->cpad[p], G.pitch, B->probs[p].c, G.n2, dsize(G.dtype),
                                         (int64_t)G.n0 * G.n1, G.n2, s));
    }
    if (B->d_bar) HIPCHK(fdw::launch_zero(B->d_bar, sizeof(unsigned) * fdw::kProgressWords, s));
    if (B->timed) HIPCHK(hipEventRecord(B->ev[0], s));
    if ((rc = plan_sweep(*B, 0, B->nfw, s))) return rc;
    if (B->timed) HIPCHK(hipEventRecord(B->ev[1], s));
    for (int p = 0; p < np; ++p) {
        const fd_problem& q = B->probs[p];
        const Geo& G = B->G[p];
        const Plan& P = B->P[p];
        if (q.acq.nrec == 0) continue;
        void *up = nullptr, *ul = nullptr;
        final_levels(B->st[p].u_a, B->st[p].u_b, q.nt, &up, &ul);
        HIPCHK(fdw::launch_terminal(G.dtype, G.acc_dtype, P.nuniq, P.d_ucell, P.d_uoff, P.d_uidx, P.d_ushot, 0, 1,
                                    G.ncell_pad, B->cp[p], 0, q.dt * q.dt, ul, up, B->st[p].acc,
                                    (const char*)B->st[p].residual +
                                        (size_t)(q.nt - 1) * q.acq.nrec * dsize(G.dtype),
                                    -q.k / q.dt, s));
    }
    if (B->timed) HIPCHK(hipEventRecord(B->ev[2], s));
    if (B->nbw > 0 && (rc = plan_sweep(*B, B->nfw, B->nbw, s))) return rc;
    if (B->timed) HIPCHK(hipEventRecord(B->ev[3], s));
    for (int p = 0; p < np; ++p) {
        const fd_problem& q = B->probs[p];
        const Geo& G = B->G[p];
        if (!B->gpad[p]) {
            HIPCHK(fdw::launch_finalize(G.dtype, G.acc_dtype, G.ncell, B->st[p].acc, q.c, 1.0 / q.k, q.grad_c, s));
        } else {   // finalise in the padded layout, then copy the rows out
            HIPCHK(fdw::launch_finalize(G.dtype, G.acc_dtype, G.ncell_pad, B->st[p].acc, B->cp[p], 1.0 / q.k,
                                        B->gpad[p], s));
            HIPCHK(fdw::launch_copy_rows(q.grad_c, G.n2, B->gpad[p], G.pitch, dsize(G.dtype),
                                         (int64_t)G.n0 * G.n1, G.n2, s));
        }
        HIPCHK(fdw::launch_sum_squares(G.dtype, B->st[p].residual, nullptr, nullptr, (int64_t)q.nt * q.acq.nrec,
                                       B->d_part, J_dev + p, s, 0.5 * q.dt));
    }
    if (B->d_bar) HIPCHK(fdw::launch_nan_if_flag(B->d_bar + 2, J_dev, np, s));
    return FD_OK;
}

int plan_timing(fd_batch_plan* B, fd_timing* t)
{
    if (!B) return fail(FD_E_ARG, "plan is null");
    if (!t) return fail(FD_E_ARG, "timing is null");
    if (!B->timed) return fail(FD_E_ARG, "the plan was made without fd_opts.timing");
    float f = 0.f, b = 0.f;
    HIPCHK(hipEventSynchronize(B->ev[3]));
    HIPCHK(hipEventElapsedTime(&f, B->ev[0], B->ev[1]));
    HIPCHK(hipEventElapsedTime(&b, B->ev[2], B->ev[3]));
    t->fwd_ms = f;
    t->fwd_launches = B->nfw;
    t->bwd_ms = b;
    t->bwd_launches = std::max(B->nbw, 0);
    t->fwd_pair_launches = t->bwd_pair_launches = 0;
    t->persistent_blocks = 0;
    if (B->d_bar) {   // word 5: the blocks that took part in the last sweep
        unsigned part = 0;
        HIPCHK(hipMemcpy(&part, B->d_bar + 5, sizeof(part), hipMemcpyDeviceToHost));
        t->persistent_blocks = (int32_t)part;
    }
    return FD_OK;
}

int plan_destroy(fd_batch_plan* B, hipStream_t s)
{
    if (!B) return FD_OK;
    for (void* p : B->owned) (void)hipFreeAsync(p, s);
    for (hipEvent_t e : B->ev)
        if (e) (void)hipEventDestroy(e);
    delete B;
    return FD_OK;
}

// Host-J form: plan, one run (captured once into a graph and launched when
// opts->graph), J copied to the host, plan released.
int batched(const fd_problem* probs, int nprob, double* J_host, const fd_opts* opts, hipStream_t s)
{
    if (!J_host) return fail(FD_E_ARG, "J_host is null");
    fd_batch_plan* B = nullptr;
    int rc = plan_create(probs, nprob, opts, s, &B);
    if (rc) return rc;
    struct Release {
        fd_batch_plan* B;
        hipStream_t s;
        ~Release() { plan_destroy(B, s); }
    } release{B, s};
    Scratch sc(s);
    double* J_dev = nullptr;
    HIPCHK(sc.get((void**)&J_dev, sizeof(double) * nprob));
    // Graph capture needs a capturable stream: the legacy null stream is not one, so a
    // graph-mode call on it works on a stream of its own (default priority), ordered
    // after the null stream's earlier work by the plan's synchronisation.
    struct OwnStream {
        hipStream_t s = nullptr;
        ~OwnStream() { if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } }
    } own;
    hipStream_t ws = s;
    if (B->G0.graph && s == nullptr) {
        HIPCHK(hipStreamCreate(&own.s));
        ws = own.s;
    }
    bool ran = false;
    if (B->G0.graph) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIPCHK(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
        const int rc2 = plan_run(B, J_dev, ws);
        hipError_t e = hipStreamEndCapture(ws, &graph);
        if (rc2) { if (graph) (void)hipGraphDestroy(graph); return rc2; }
        HIPCHK(e);
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(graph); HIPCHK(e); }
        e = hipGraphLaunch(exec, ws);
        const hipError_t e2 = hipStreamSynchronize(ws);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        HIPCHK(e);
        HIPCHK(e2);
        ran = true;
    }
    if (!ran && (rc = plan_run(B, J_dev, ws))) return rc;
    if (B->timed && (rc = plan_timing(B, B->G0.timing))) return rc;
    if (B->d_bar) {
        unsigned flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, B->d_bar + 2, sizeof(flag), hipMemcpyDeviceToHost, ws));
        HIPCHK(hipStreamSynchronize(ws));
        if (flag != 0)
            return fail(FD_E_DEVICE, "persistent launch: a wait for the launch's other blocks or for "
                                     "neighbouring groups timed out (barrier_timeout_us is shorter "
                                     "than a group's step); the results are invalid");
    }
    HIPCHK(hipMemcpyAsync(J_host, J_dev, sizeof(double) * nprob, hipMemcpyDeviceToHost, ws));
    HIPCHK(hipStreamSynchronize(ws));
    for (int p = 0; p < nprob; ++p)
        if (!std::isfinite(J_host[p]))
            return fail(FD_E_NONFINITE, "problem " + std::to_string(p) + ": misfit is not finite");
    return FD_OK;
}

}  // namespace

extern "C" {

int fd_adjoint_sensitivity_batched(const fd_problem* probs, int32_t nprob, double* J_host,
                                   const fd_opts* opts, void* stream)
{
    g_err.clear();
    return batched(probs, nprob, J_host, opts, (hipStream_t)stream);
}

int fd_batch_plan_create(const fd_problem* probs, int32_t nprob, const fd_opts* opts, void* stream,
                         fd_batch_plan** plan)
{
    g_err.clear();
    return plan_create(probs, nprob, opts, (hipStream_t)stream, plan);
}

int fd_batch_run(fd_batch_plan* plan, double* J, void* stream)
{
    g_err.clear();
    return plan_run(plan, J, (hipStream_t)stream);
}

int fd_batch_timing(fd_batch_plan* plan, fd_timing* timing)
{
    g_err.clear();
    return plan_timing(plan, timing);
}

int fd_batch_plan_destroy(fd_batch_plan* plan, void* stream)
{
    g_err.clear();
    return plan_destroy(plan, (hipStream_t)stream);
}

}  // extern "C"
