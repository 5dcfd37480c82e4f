// fdwave C-ABI: argument validation, CFL check, block plans, device scratch and the
// time loops of the paper's Algorithm 1 (forward sweep, terminal hand-over,
// superposed backward sweep, finalisation).  Kernels live in fdw_kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdwave.h"
#include "fdw_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

// Textbook central second-derivative weights a_1..a_r (orders 2, 4, 8).
const double kW2[1] = {1.0};
const double kW4[2] = {4.0 / 3.0, -1.0 / 12.0};
const double kW8[4] = {8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

const double* weights(int order)
{
    return order == 2 ? kW2 : order == 4 ? kW4 : order == 8 ? kW8 : nullptr;
}

size_t dsize(int dtype) { return dtype == FD_F64 ? 8 : 4; }

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? FD_E_NOMEM : FD_E_DEVICE,               \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

// The pointer must lie in a device allocation that covers `bytes` from it.
int check_dev(const void* p, size_t bytes, const char* what)
{
    if (bytes == 0) return FD_OK;
    if (!p) return fail(FD_E_ARG, std::string(what) + " is null");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess || base == nullptr) {
        (void)hipGetLastError();
        return fail(FD_E_ARG, std::string(what) + " is not a device allocation");
    }
    const char* b = (const char*)base;
    const char* q = (const char*)p;
    if (q < b || (size_t)(q - b) + bytes > size)
        return fail(FD_E_ARG, std::string(what) + " is smaller than required (" +
                                  std::to_string(bytes) + " bytes)");
    return FD_OK;
}

struct Geo {
    fd_timing* timing = nullptr;
    int ndim, r, dtype, acc_dtype, variant;
    int chunk = 0;       // requested planes per block (0: library choice)
    int n0, n1, n2;      // internal extents (2D: n1 = 1)
    int64_t ncell;
    double dx, inv_vol;
};

int check_grid(const fd_grid* g, const fd_opts* o, Geo* out)
{
    if (!g) return fail(FD_E_ARG, "grid is null");
    if (g->ndim != 2 && g->ndim != 3) return fail(FD_E_ARG, "ndim must be 2 or 3");
    if (!weights(g->order)) return fail(FD_E_ARG, "order must be 2, 4 or 8");
    if (g->dtype != FD_F32 && g->dtype != FD_F64) return fail(FD_E_ARG, "dtype must be FD_F32 or FD_F64");
    if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(FD_E_ARG, "dx must be positive and finite");
    const int r = g->order / 2;
    int64_t n[3] = {g->shape[0], g->shape[1], g->ndim == 3 ? g->shape[2] : 1};
    for (int ax = 0; ax < g->ndim; ++ax) {
        if (n[ax] < r) return fail(FD_E_ARG, "every extent must be >= order/2");
        if (n[ax] > (1 << 30)) return fail(FD_E_ARG, "extent too large");
    }
    if (n[1] * n[2] >= ((int64_t)1 << 31)) return fail(FD_E_ARG, "plane normal to axis 0 too large");
    Geo G;
    G.ndim = g->ndim;
    G.r = r;
    G.dtype = g->dtype;
    G.acc_dtype = FD_F64;
    G.variant = g->ndim == 3 ? 3 : 1;   // measured best default tile (64 x 8 in 3D)
    if (o) {
        if (o->acc_dtype != FD_F32 && o->acc_dtype != FD_F64)
            return fail(FD_E_ARG, "acc_dtype must be FD_F32 or FD_F64");
        G.acc_dtype = o->acc_dtype;
        if (o->variant != 0) {
            if (o->variant < 1 || o->variant > fdw::variant_count(g->ndim))
                return fail(FD_E_ARG, "variant out of range");
            G.variant = o->variant;
        }
        G.timing = o->timing;
        if (o->chunk < 0) return fail(FD_E_ARG, "chunk is negative");
        G.chunk = o->chunk;
    }
    if (G.dtype == FD_F64) G.acc_dtype = FD_F64;
    G.n0 = (int)n[0];
    if (g->ndim == 3) { G.n1 = (int)n[1]; G.n2 = (int)n[2]; }
    else { G.n1 = 1; G.n2 = (int)n[1]; }
    G.ncell = n[0] * n[1] * n[2];
    G.dx = g->dx;
    G.inv_vol = 1.0 / std::pow(g->dx, (double)g->ndim);
    *out = G;
    return FD_OK;
}

int check_cells(int count, const int64_t* cells, int64_t ncell, const char* what)
{
    if (count < 0) return fail(FD_E_ARG, std::string(what) + " count is negative");
    if (count > 0 && !cells) return fail(FD_E_ARG, std::string(what) + " cells are null");
    for (int i = 0; i < count; ++i)
        if (cells[i] < 0 || cells[i] >= ncell)
            return fail(FD_E_ARG, std::string(what) + " cell " + std::to_string(i) + " out of range");
    return FD_OK;
}

int check_acq(const fd_acq* a, const Geo& G, int nt)
{
    if (!a) return fail(FD_E_ARG, "acq is null");
    int rc = check_cells(a->nsrc, a->src_cell, G.ncell, "source");
    if (rc) return rc;
    rc = check_cells(a->nrec, a->rec_cell, G.ncell, "receiver");
    if (rc) return rc;
    return check_dev(a->wavelet, (size_t)nt * a->nsrc * dsize(G.dtype), "wavelet");
}

// Device scratch taken stream-ordered and released at scope exit.
struct Scratch {
    hipStream_t s;
    std::vector<void*> ptrs;
    explicit Scratch(hipStream_t st) : s(st) {}
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFreeAsync(p, s);
    }
    hipError_t get(void** p, size_t bytes)
    {
        *p = nullptr;
        if (bytes == 0) bytes = 8;
        hipError_t e = hipMallocAsync(p, bytes, s);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

// Host statistics of the speed field: max, min, non-finite count.
int speed_stats(const Geo& G, const void* c, hipStream_t s, Scratch& sc, double* cmax, double* cmin)
{
    void* part = nullptr;
    void* out = nullptr;
    HIPCHK(sc.get(&part, sizeof(double) * 3 * fdw::kReduceBlocks));
    HIPCHK(sc.get(&out, sizeof(double) * 3));
    HIPCHK(fdw::launch_speed_stats(G.dtype, c, G.ncell, (double*)out, (double*)part, s));
    double h[3];
    HIPCHK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[2] > 0) return fail(FD_E_NONFINITE, "speed field has non-finite entries");
    if (!(h[1] > 0.0)) return fail(FD_E_NONFINITE, "speed field must be positive");
    *cmax = h[0];
    *cmin = h[1];
    return FD_OK;
}

double cfl_limit(int ndim, int order)
{
    const double* a = weights(order);
    if (!a || (ndim < 1 || ndim > 3)) return 0.0;
    const int r = order / 2;
    double a0 = 0.0, sym = 0.0;
    for (int j = 1; j <= r; ++j) a0 -= 2.0 * a[j - 1];
    sym = a0;
    for (int j = 1; j <= r; ++j) sym += 2.0 * a[j - 1] * ((j & 1) ? -1.0 : 1.0);
    return 2.0 / std::sqrt(ndim * std::fabs(sym));
}

int check_cfl(const Geo& G, double cmax, double dt)
{
    const double courant = cmax * dt / G.dx;
    const double lim = cfl_limit(G.ndim, 2 * G.r);
    if (courant > lim * (1.0 + 1e-12)) {
        char buf[160];
        snprintf(buf, sizeof buf, "Courant number %.6g exceeds the stability limit %.6g", courant, lim);
        return fail(FD_E_CFL, buf);
    }
    return FD_OK;
}

// Block decomposition plus the per-block event lists of sources and receivers.
struct Plan {
    fdw::Variant v;
    int nty, ntz, nch, chunk, nblk;
    int32_t* d_off = nullptr;
    fdw::Event* d_ev = nullptr;
    // distinct receiver cells (terminal hand-over)
    int nuniq = 0;
    int64_t* d_ucell = nullptr;
    int32_t* d_uoff = nullptr;
    int32_t* d_uidx = nullptr;
};

int make_plan(const Geo& G, const fd_acq* acq, bool want_uniq, hipStream_t s, Scratch& sc, Plan* P)
{
    fdw::Variant v = fdw::variant_shape(G.ndim, G.variant);
    if (v.tz == 0) return fail(FD_E_ARG, "invalid variant");
    P->v = v;
    P->ntz = (G.n2 + v.tz - 1) / v.tz;
    P->nty = (G.n1 + v.ty - 1) / v.ty;
    const int64_t tiles = (int64_t)P->ntz * P->nty;
    if (G.chunk > 0) {
        P->chunk = std::min(G.chunk, G.n0);
    } else {
        // split axis 0 so that the launch holds ~4M threads (several rounds of resident
        // blocks: a short last round leaves the chip idle), keeping chunks >= 16 r
        // planes in 3D (each chunk re-reads 2r planes to fill its queue)
        const int64_t want_blocks = ((int64_t)4 << 20) / v.threads;
        const int64_t want = (want_blocks + tiles - 1) / tiles;
        const int min_chunk = G.ndim == 3 ? 16 * G.r : 2 * G.r;
        const int64_t maxch = std::max<int64_t>(1, G.n0 / min_chunk);
        const int64_t nch = std::max<int64_t>(1, std::min(want, maxch));
        P->chunk = (int)((G.n0 + nch - 1) / nch);
    }
    P->nch = (G.n0 + P->chunk - 1) / P->chunk;
    const int64_t nblk = tiles * P->nch;
    if (nblk > (1 << 28)) return fail(FD_E_ARG, "grid too large for the block decomposition");
    P->nblk = (int)nblk;

    struct Item { int64_t key; fdw::Event e; };
    std::vector<Item> items;
    const int nsrc = acq ? acq->nsrc : 0;
    const int nrec = acq ? acq->nrec : 0;
    items.reserve(nsrc + nrec);
    auto add = [&](int64_t cell, int kind, int idx) {
        const int64_t plane = (int64_t)G.n1 * G.n2;
        const int x = (int)(cell / plane);
        const int64_t rem = cell - (int64_t)x * plane;
        const int y = (int)(rem / G.n2);
        const int z = (int)(rem - (int64_t)y * G.n2);
        const int ty = y / v.ty, tz = z / v.tz, ch = x / P->chunk;
        const int64_t b = ((int64_t)ch * P->nty + ty) * P->ntz + tz;
        fdw::Event e;
        e.plane = x;
        e.lane = (y - ty * v.ty) * v.tz + (z - tz * v.tz);
        e.kind = kind;
        e.idx = idx;
        items.push_back({b, e});
    };
    for (int i = 0; i < nsrc; ++i) add(acq->src_cell[i], fdw::EV_SRC, i);
    for (int i = 0; i < nrec; ++i) add(acq->rec_cell[i], fdw::EV_REC, i);
    std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.e.plane != b.e.plane) return a.e.plane < b.e.plane;
        if (a.e.lane != b.e.lane) return a.e.lane < b.e.lane;
        if (a.e.kind != b.e.kind) return a.e.kind < b.e.kind;
        return a.e.idx < b.e.idx;
    });
    std::vector<int32_t> off(P->nblk + 1, 0);
    std::vector<fdw::Event> ev(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        off[items[i].key + 1]++;
        ev[i] = items[i].e;
    }
    for (int b = 0; b < P->nblk; ++b) off[b + 1] += off[b];

    HIPCHK(sc.get((void**)&P->d_off, sizeof(int32_t) * off.size()));
    HIPCHK(sc.get((void**)&P->d_ev, sizeof(fdw::Event) * std::max<size_t>(1, ev.size())));
    HIPCHK(hipMemcpyAsync(P->d_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, s));
    if (!ev.empty())
        HIPCHK(hipMemcpyAsync(P->d_ev, ev.data(), sizeof(fdw::Event) * ev.size(), hipMemcpyHostToDevice, s));

    if (want_uniq && nrec > 0) {
        std::vector<std::pair<int64_t, int32_t>> rc(nrec);
        for (int i = 0; i < nrec; ++i) rc[i] = {acq->rec_cell[i], i};
        std::sort(rc.begin(), rc.end());
        std::vector<int64_t> ucell;
        std::vector<int32_t> uoff{0}, uidx(nrec);
        for (int i = 0; i < nrec; ++i) {
            if (i == 0 || rc[i].first != rc[i - 1].first) {
                if (i) uoff.push_back(i);
                ucell.push_back(rc[i].first);
            }
            uidx[i] = rc[i].second;
        }
        uoff.push_back(nrec);
        P->nuniq = (int)ucell.size();
        HIPCHK(sc.get((void**)&P->d_ucell, sizeof(int64_t) * ucell.size()));
        HIPCHK(sc.get((void**)&P->d_uoff, sizeof(int32_t) * uoff.size()));
        HIPCHK(sc.get((void**)&P->d_uidx, sizeof(int32_t) * uidx.size()));
        HIPCHK(hipMemcpyAsync(P->d_ucell, ucell.data(), sizeof(int64_t) * ucell.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_uoff, uoff.data(), sizeof(int32_t) * uoff.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_uidx, uidx.data(), sizeof(int32_t) * uidx.size(), hipMemcpyHostToDevice, s));
    }
    // the host vectors die with this frame: finish the copies first
    HIPCHK(hipStreamSynchronize(s));
    return FD_OK;
}

fdw::StepArgs base_args(const Geo& G, const Plan& P, const void* c, double dt)
{
    fdw::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = c;
    a.n0 = G.n0; a.n1 = G.n1; a.n2 = G.n2;
    const double* w = weights(2 * G.r);
    for (int j = 0; j < G.r; ++j) a.w[j] = w[j] / (G.dx * G.dx);
    a.dt2 = dt * dt;
    a.inv_vol = G.inv_vol;
    a.blk_off = P.d_off;
    a.ev = P.d_ev;
    a.nty = P.nty; a.ntz = P.ntz; a.chunk_len = P.chunk; a.nblk = P.nblk;
    return a;
}

int step(const Geo& G, const Plan& P, const fdw::StepArgs& a, hipStream_t s)
{
    HIPCHK(fdw::launch_step(G.ndim, G.r, G.dtype, G.acc_dtype, G.variant, P.nblk, a, s));
    return FD_OK;
}

int check_time(double dt, int nt)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FD_E_ARG, "dt must be positive and finite");
    if (nt < 1) return fail(FD_E_ARG, "nt must be >= 1");
    return FD_OK;
}

// HIP events around the step launches of one sweep (only when a timing record is asked for).
struct SweepTimer {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    hipStream_t s;
    SweepTimer(bool want, hipStream_t st) : on(want), s(st)
    {
        if (on && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) on = false;
    }
    ~SweepTimer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start() { if (on) (void)hipEventRecord(a, s); }
    void stop() { if (on) (void)hipEventRecord(b, s); }
    // waits for the second event; returns milliseconds (0 when off)
    double ms()
    {
        float t = 0.f;
        if (!on || hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess)
            return 0.0;
        return (double)t;
    }
};

// Validation shared by the sweeps: grid, acquisition, time axis, speed, CFL.
int prepare(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
            const fd_opts* opts, hipStream_t s, Scratch& sc, Geo* G, bool stats)
{
    int rc = check_grid(grid, opts, G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if ((rc = check_acq(acq, *G, nt))) return rc;
    if ((rc = check_dev(c, G->ncell * dsize(G->dtype), "c"))) return rc;
    if (stats) {
        double cmax, cmin;
        if ((rc = speed_stats(*G, c, s, sc, &cmax, &cmin))) return rc;
        if ((rc = check_cfl(*G, cmax, dt))) return rc;
    }
    return FD_OK;
}

int forward_sweep(const Geo& G, const Plan& P, const void* c, const fd_acq* acq, double dt, int nt,
                  const void* obs, void* ua, void* ub, void* acc, void* resid, void* traces,
                  hipStream_t s)
{
    const size_t fb = G.ncell * dsize(G.dtype);
    HIPCHK(hipMemsetAsync(ua, 0, fb, s));
    HIPCHK(hipMemsetAsync(ub, 0, fb, s));
    if (acc) HIPCHK(hipMemsetAsync(acc, 0, G.ncell * dsize(G.acc_dtype), s));
    fdw::StepArgs a = base_args(G, P, c, dt);
    a.acc = acc;
    a.wavelet = acq->wavelet;
    a.nsrc = acq->nsrc;
    a.sample = 1;
    a.traces = traces;
    a.resid = resid;
    a.obs = obs;
    a.nrec = acq->nrec;
    void* prev = ua;   // level n-1
    void* cur = ub;    // level n
    SweepTimer tm(G.timing != nullptr, s);
    tm.start();
    for (int n = 0; n < nt; ++n) {
        a.ucur = cur;
        a.unew = prev;
        a.acc_sign = (acc && n < nt - 1) ? 1 : 0;   // the last interval is settled at hand-over
        a.row_src = n;
        a.row_rec = n;
        int rc = step(G, P, a, s);
        if (rc) return rc;
        std::swap(prev, cur);
    }
    tm.stop();
    if (G.timing) {
        G.timing->fwd_ms = tm.ms();
        G.timing->fwd_launches = nt;
    }
    return FD_OK;
}

// After forward_sweep from (ua, ub): the buffers holding u^{nt-1} and u^nt.
void final_levels(void* ua, void* ub, int nt, void** prev, void** cur)
{
    if (nt & 1) { *cur = ua; *prev = ub; }
    else { *cur = ub; *prev = ua; }
}

int backward_sweep(const Geo& G, const Plan& P, const void* c, const fd_acq* acq, double dt, int nt,
                   double k, void* ua, void* ub, void* acc, void* resid, hipStream_t s)
{
    void* up = nullptr;   // u^{nt-1} -> v^{nt-1}
    void* ul = nullptr;   // u^nt = v^nt
    final_levels(ua, ub, nt, &up, &ul);
    const double rec_scale = -k / dt;   // k fdag^n = -(k/dt) residual^n
    if (acq->nrec > 0)
        HIPCHK(fdw::launch_terminal(G.dtype, G.acc_dtype, P.nuniq, P.d_ucell, P.d_uoff, P.d_uidx, c,
                                    dt * dt, ul, up, acc,
                                    (const char*)resid + (size_t)(nt - 1) * acq->nrec * dsize(G.dtype),
                                    rec_scale, s));
    fdw::StepArgs a = base_args(G, P, c, dt);
    a.acc = acc;
    a.acc_sign = -1;
    a.wavelet = acq->wavelet;
    a.nsrc = acq->nsrc;
    a.inject_rec = 1;
    a.resid = resid;
    a.nrec = acq->nrec;
    a.rec_scale = rec_scale;
    void* vj = up;    // v^j
    void* vn = ul;    // v^{j+1}, overwritten by v^{j-1}
    SweepTimer tm(G.timing != nullptr && nt > 1, s);
    tm.start();
    for (int j = nt - 1; j >= 1; --j) {
        a.ucur = vj;
        a.unew = vn;
        a.row_src = j;
        a.row_rec = j - 1;
        int rc = step(G, P, a, s);
        if (rc) return rc;
        std::swap(vj, vn);
    }
    tm.stop();
    if (G.timing) {
        G.timing->bwd_ms = tm.ms();
        G.timing->bwd_launches = nt - 1;
    }
    return FD_OK;
}

int misfit_sum(int dtype, const void* x, const void* y, void* diff, int64_t n, hipStream_t s,
               Scratch& sc, double* out)
{
    void* part = nullptr;
    void* dout = nullptr;
    HIPCHK(sc.get(&part, sizeof(double) * fdw::kReduceBlocks));
    HIPCHK(sc.get(&dout, sizeof(double)));
    HIPCHK(fdw::launch_sum_squares(dtype, x, y, diff, n, (double*)part, (double*)dout, s));
    HIPCHK(hipMemcpyAsync(out, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FD_OK;
}

int check_state(const fd_state* st, const Geo& G, int nt, int nrec)
{
    if (!st) return fail(FD_E_ARG, "state is null");
    const size_t fb = G.ncell * dsize(G.dtype);
    int rc;
    if ((rc = check_dev(st->u_a, fb, "state.u_a"))) return rc;
    if ((rc = check_dev(st->u_b, fb, "state.u_b"))) return rc;
    if ((rc = check_dev(st->acc, G.ncell * dsize(G.acc_dtype), "state.acc"))) return rc;
    if ((rc = check_dev(st->residual, (size_t)nt * nrec * dsize(G.dtype), "state.residual"))) return rc;
    return FD_OK;
}

// `own_state`: the state arrays were allocated by the library itself in this call.
int sens_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
                 const void* observed, const fd_state* st, void* traces, double* J_host,
                 const fd_opts* opts, hipStream_t s, bool own_state)
{
    Scratch sc(s);
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, true);
    if (rc) return rc;
    if (!own_state && (rc = check_state(st, G, nt, acq->nrec))) return rc;
    const size_t tb = (size_t)nt * acq->nrec * dsize(G.dtype);
    if ((rc = check_dev(observed, tb, "observed"))) return rc;
    if (traces && (rc = check_dev(traces, tb, "traces"))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    if ((rc = forward_sweep(G, P, c, acq, dt, nt, observed, st->u_a, st->u_b, st->acc, st->residual,
                            traces, s)))
        return rc;
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
                  bool own_state)
{
    Scratch sc(s);
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, false);
    if (rc) return rc;
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    if (!std::isfinite(grad_scale)) return fail(FD_E_ARG, "grad_scale must be finite");
    if (!own_state && (rc = check_state(st, G, nt, acq->nrec))) return rc;
    if ((rc = check_dev(grad, G.ncell * dsize(G.dtype), "grad_c"))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, true, s, sc, &P))) return rc;
    if ((rc = backward_sweep(G, P, c, acq, dt, nt, k, st->u_a, st->u_b, st->acc, st->residual, s)))
        return rc;
    HIPCHK(fdw::launch_finalize(G.dtype, G.acc_dtype, G.ncell, st->acc, c, grad_scale / k, grad, s));
    return FD_OK;
}

}  // namespace

extern "C" {

const char* fd_last_error(void) { return g_err.c_str(); }

double fd_cfl_limit(int32_t ndim, int32_t order) { return cfl_limit(ndim, order); }

int32_t fd_variant_count(int32_t ndim)
{
    return (ndim == 2 || ndim == 3) ? fdw::variant_count(ndim) : 0;
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
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    void *ua = nullptr, *ub = nullptr;
    HIPCHK(sc.get(&ua, G.ncell * dsize(G.dtype)));
    HIPCHK(sc.get(&ub, G.ncell * dsize(G.dtype)));
    return forward_sweep(G, P, c, acq, dt, nt, nullptr, ua, ub, nullptr, nullptr, traces, s);
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
    hipStream_t s = (hipStream_t)stream;
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if (!acq) return fail(FD_E_ARG, "acq is null");
    if (acq->nrec < 0) return fail(FD_E_ARG, "receiver count is negative");
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    Scratch sc(s);
    fd_state st;
    HIPCHK(sc.get(&st.u_a, G.ncell * dsize(G.dtype)));
    HIPCHK(sc.get(&st.u_b, G.ncell * dsize(G.dtype)));
    HIPCHK(sc.get(&st.acc, G.ncell * dsize(G.acc_dtype)));
    HIPCHK(sc.get(&st.residual, (size_t)nt * acq->nrec * dsize(G.dtype)));
    if ((rc = sens_forward(grid, c, acq, dt, nt, observed, &st, traces_or_null, J_host, opts, s, true)))
        return rc;
    return sens_backward(grid, c, acq, dt, nt, k, &st, 1.0, grad_c, opts, s, true);
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
        if ((rc = step(G, P, a, s))) return rc;
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
