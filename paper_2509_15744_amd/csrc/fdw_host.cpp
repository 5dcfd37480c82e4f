// fdwave host runtime shared by the entry points (declared in fdw_host.h): argument
// validation, CFL check, block plans with per-block event lists, device scratch and
// the time loops of the paper's Algorithm 1 (forward sweep with K(u,u), superposed
// backward sweep with K(v,v)).

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "fdw_aux.h"
#include "fdw_host.h"

namespace fdh {

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
    G.variant = 1;   // one cell per lane: valid for every extent
    if (o) {
        if (o->acc_dtype != FD_F32 && o->acc_dtype != FD_F64)
            return fail(FD_E_ARG, "acc_dtype must be FD_F32 or FD_F64");
        G.acc_dtype = o->acc_dtype;
        if (o->variant != 0) {
            if (o->variant < 1 || o->variant > fdw::variant_count(g->ndim))
                return fail(FD_E_ARG, "variant out of range");
            G.variant = o->variant;
            G.auto_variant = false;
        }
        G.timing = o->timing;
        if (o->chunk < 0) return fail(FD_E_ARG, "chunk is negative");
        G.chunk = o->chunk;
        if (o->max_group != 0 && o->max_group != 1 && o->max_group != 2 && o->max_group != 4)
            return fail(FD_E_ARG, "max_group must be 0, 1, 2 or 4");
        G.max_group = o->max_group;
        G.graph = o->graph;
        G.persistent = o->persistent;
        if (o->barrier_timeout_us < 0) return fail(FD_E_ARG, "barrier_timeout_us is negative");
        G.barrier_timeout_us = o->barrier_timeout_us;
        if (o->variant_plain < 0 || o->variant_plain > fdw::variant_count(g->ndim))
            return fail(FD_E_ARG, "variant_plain out of range");
        if (o->chunk_plain < 0) return fail(FD_E_ARG, "chunk_plain is negative");
        G.variant_plain = o->variant_plain;
        G.chunk_plain = o->chunk_plain;
        G.no_partials = o->no_partials != 0;
        if (o->pairs < -1 || o->pairs > 1) return fail(FD_E_ARG, "pairs must be -1, 0 or 1");
        G.pairs = o->pairs;
    }
    if (G.dtype == FD_F64) G.acc_dtype = FD_F64;
    G.n0 = (int)n[0];
    if (g->ndim == 3) { G.n1 = (int)n[1]; G.n2 = (int)n[2]; }
    else { G.n1 = 1; G.n2 = (int)n[1]; }
    G.ncell = n[0] * n[1] * n[2];
    G.pitch = G.n2;
    G.ncell_pad = G.ncell;
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

int nshots(const fd_acq* a) { return a->nshot > 1 ? a->nshot : 1; }

int check_tags(int count, const int32_t* tags, int nshot, const char* what)
{
    if (nshot <= 1 || count == 0) return FD_OK;
    if (!tags) return fail(FD_E_ARG, std::string(what) + " shot tags are null");
    for (int i = 0; i < count; ++i)
        if (tags[i] < 0 || tags[i] >= nshot)
            return fail(FD_E_ARG, std::string(what) + " " + std::to_string(i) + " has a shot out of range");
    return FD_OK;
}

int check_acq(const fd_acq* a, const Geo& G, int nt)
{
    if (!a) return fail(FD_E_ARG, "acq is null");
    if (a->nshot < 0) return fail(FD_E_ARG, "nshot is negative");
    int rc = check_cells(a->nsrc, a->src_cell, G.ncell, "source");
    if (rc) return rc;
    rc = check_cells(a->nrec, a->rec_cell, G.ncell, "receiver");
    if (rc) return rc;
    if ((rc = check_tags(a->nsrc, a->src_shot, a->nshot, "source"))) return rc;
    if ((rc = check_tags(a->nrec, a->rec_shot, a->nshot, "receiver"))) return rc;
    return check_dev(a->wavelet, (size_t)nt * a->nsrc * dsize(G.dtype), "wavelet");
}

int src_shot(const fd_acq* a, int i) { return a->nshot > 1 ? a->src_shot[i] : 0; }
int rec_shot(const fd_acq* a, int i) { return a->nshot > 1 ? a->rec_shot[i] : 0; }

double cfl_limit(int ndim, int order)
{
    const double* a = weights(order);
    if (!a || (ndim < 1 || ndim > 3)) return 0.0;
    const int r = order / 2;
    double a0 = 0.0;
    for (int j = 1; j <= r; ++j) a0 -= 2.0 * a[j - 1];
    double sym = a0;
    for (int j = 1; j <= r; ++j) sym += 2.0 * a[j - 1] * ((j & 1) ? -1.0 : 1.0);
    return 2.0 / std::sqrt(ndim * std::fabs(sym));
}

// Speed statistics of several fields with one synchronisation: each gets max, min and
// a non-finite count; then the positivity, finiteness and CFL checks.
int check_speeds(const std::vector<const Geo*>& geos, const std::vector<const void*>& cs,
                 const std::vector<double>& dts, hipStream_t s, Scratch& sc)
{
    const size_t m = geos.size();
    void* part = nullptr;
    void* out = nullptr;
    HIPCHK(sc.get(&part, sizeof(double) * 3 * fdw::kReduceBlocks));
    HIPCHK(sc.get(&out, sizeof(double) * 3 * m));
    std::vector<double> h(3 * m);
    for (size_t i = 0; i < m; ++i)
        HIPCHK(fdw::launch_speed_stats(geos[i]->dtype, cs[i], geos[i]->ncell, (double*)out + 3 * i,
                                       (double*)part, s));
    HIPCHK(hipMemcpyAsync(h.data(), out, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t i = 0; i < m; ++i) {
        const std::string who = m > 1 ? "problem " + std::to_string(i) + ": " : "";
        if (h[3 * i + 2] > 0) return fail(FD_E_NONFINITE, who + "speed field has non-finite entries");
        if (!(h[3 * i + 1] > 0.0)) return fail(FD_E_NONFINITE, who + "speed field must be positive");
        const Geo& G = *geos[i];
        const double courant = h[3 * i] * dts[i] / G.dx;
        const double lim = cfl_limit(G.ndim, 2 * G.r);
        if (courant > lim * (1.0 + 1e-12)) {
            char buf[200];
            snprintf(buf, sizeof buf, "%sCourant number %.6g exceeds the stability limit %.6g",
                     who.c_str(), courant, lim);
            return fail(FD_E_CFL, buf);
        }
    }
    return FD_OK;
}

// `pairs`: one group per shot carrying two fields, the shot's wavefield in slot 0 (its
// sources inject there) and its adjoint field in slot 1 (its receivers inject there).
int make_plan(Geo& G, const fd_acq* acq, bool want_uniq, hipStream_t s, Scratch& sc, Plan* P,
              bool pairs)
{
    if (G.auto_variant) apply_tuned(G, acq ? nshots(acq) : 1);
    fdw::Variant v = fdw::variant_shape(G.ndim, G.variant);
    if (v.tz == 0) return fail(FD_E_ARG, "invalid variant");
    if (pairs && v.max_shots < 2)
        return fail(FD_E_ARG, "variant " + std::to_string(G.variant) + " cannot carry two fields per launch");
    if (G.n2 % v.vz != 0)
        return fail(FD_E_ARG, "variant " + std::to_string(G.variant) +
                                  " needs the contiguous extent to be a multiple of " + std::to_string(v.vz));
    P->v = v;
    P->variant = G.variant;
    P->ntz = (G.n2 + v.tz - 1) / v.tz;
    P->nty = (G.n1 + v.ty - 1) / v.ty;
    const int64_t tiles = (int64_t)P->ntz * P->nty;
    if (G.chunk > 0) {
        P->chunk = std::min(G.chunk, G.n0);
    } else {
        // split axis 0 so that the launch holds ~4M threads (several rounds of resident
        // blocks: a short last round leaves the chip idle), keeping chunks >= 16 r
        // planes in 3D (each chunk re-reads 2r planes to fill its queue); in 2D short
        // chunks win (a block's march serialises its rows), down to 4 rows
        const int64_t want_blocks = ((int64_t)4 << 20) / v.threads;
        const int64_t want = (want_blocks + tiles - 1) / tiles;
        const int min_chunk = G.ndim == 3 ? 16 * G.r : std::min(2 * G.r, 4);
        const int64_t maxch = std::max<int64_t>(1, G.n0 / min_chunk);
        const int64_t nch = std::max<int64_t>(1, std::min(want, maxch));
        P->chunk = (int)((G.n0 + nch - 1) / nch);
    }
    P->nch = (G.n0 + P->chunk - 1) / P->chunk;
    const int64_t nblk = tiles * P->nch;
    if (nblk > (1 << 28)) return fail(FD_E_ARG, "grid too large for the block decomposition");
    P->nblk = (int)nblk;

    // shot groups: sizes 4, 2, 1 up to the variant's (and the caller's) largest
    const int ns = acq ? nshots(acq) : 1;
    int gmax = v.max_shots;
    if (G.max_group > 0) gmax = std::min(gmax, G.max_group);
    for (int g0 = 0; g0 < ns;) {
        int sz = 4;
        while (sz > gmax || g0 + sz > ns) sz >>= 1;
        Group gr;
        gr.g0 = g0;
        gr.size = pairs ? 2 : sz;
        P->groups.push_back(gr);
        g0 += pairs ? 1 : sz;
    }

    const int nsrc = acq ? acq->nsrc : 0;
    const int nrec = acq ? acq->nrec : 0;
    std::vector<std::vector<int32_t>> offs;
    std::vector<std::vector<fdw::EvPlane>> grps;
    std::vector<std::vector<fdw::Event>> evs;
    for (Group& gr : P->groups) {
        struct Item { int64_t key; fdw::Event e; };
        std::vector<Item> items;
        auto add = [&](int64_t cell, int kind, int idx, int shot) {
            int slot = shot - gr.g0;
            if (pairs) {
                if (shot != gr.g0) return;
                slot = kind == fdw::EV_REC ? 1 : 0;
            } else if (shot < gr.g0 || shot >= gr.g0 + gr.size) {
                return;
            }
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
            e.kind = kind | (slot << 1);
            e.idx = idx;
            items.push_back({b, e});
        };
        for (int i = 0; i < nsrc; ++i) add(acq->src_cell[i], fdw::EV_SRC, i, src_shot(acq, i));
        for (int i = 0; i < nrec; ++i) add(acq->rec_cell[i], fdw::EV_REC, i, rec_shot(acq, i));
        std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
            if (a.key != b.key) return a.key < b.key;
            if (a.e.plane != b.e.plane) return a.e.plane < b.e.plane;
            if (a.e.lane != b.e.lane) return a.e.lane < b.e.lane;
            if (a.e.kind != b.e.kind) return a.e.kind < b.e.kind;
            return a.e.idx < b.e.idx;
        });
        // plane groups: runs of one block's events in one plane
        std::vector<int32_t> off(P->nblk + 1, 0);
        std::vector<fdw::EvPlane> grp;
        std::vector<fdw::Event> ev(items.size());
        for (size_t i = 0; i < items.size(); ++i) {
            ev[i] = items[i].e;
            if (i == 0 || items[i].key != items[i - 1].key || ev[i].plane != ev[i - 1].plane) {
                fdw::EvPlane g;
                g.plane = ev[i].plane;
                g.begin = (int32_t)i;
                g.end = (int32_t)i;
                g.pad = 0;
                grp.push_back(g);
                off[items[i].key + 1]++;
            }
            grp.back().end = (int32_t)i + 1;
        }
        for (int b = 0; b < P->nblk; ++b) off[b + 1] += off[b];
        HIPCHK(sc.get((void**)&gr.d_off, sizeof(int32_t) * off.size()));
        HIPCHK(sc.get((void**)&gr.d_grp, sizeof(fdw::EvPlane) * std::max<size_t>(1, grp.size())));
        HIPCHK(sc.get((void**)&gr.d_ev, sizeof(fdw::Event) * std::max<size_t>(1, ev.size())));
        HIPCHK(hipMemcpyAsync(gr.d_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, s));
        if (!grp.empty())
            HIPCHK(hipMemcpyAsync(gr.d_grp, grp.data(), sizeof(fdw::EvPlane) * grp.size(), hipMemcpyHostToDevice, s));
        if (!ev.empty())
            HIPCHK(hipMemcpyAsync(gr.d_ev, ev.data(), sizeof(fdw::Event) * ev.size(), hipMemcpyHostToDevice, s));
        offs.push_back(std::move(off));
        grps.push_back(std::move(grp));
        evs.push_back(std::move(ev));
    }

    std::vector<int64_t> ucell;
    std::vector<int32_t> uoff, uidx, ushot;
    if (want_uniq && nrec > 0) {
        struct R { int64_t cell; int32_t shot, idx; };
        std::vector<R> rc(nrec);
        for (int i = 0; i < nrec; ++i) rc[i] = {acq->rec_cell[i], rec_shot(acq, i), i};
        std::sort(rc.begin(), rc.end(), [](const R& a, const R& b) {
            if (a.cell != b.cell) return a.cell < b.cell;
            if (a.shot != b.shot) return a.shot < b.shot;
            return a.idx < b.idx;
        });
        uoff.push_back(0);
        for (int i = 0; i < nrec; ++i) {
            if (i == 0 || rc[i].cell != rc[i - 1].cell) {
                if (i) uoff.push_back(i);
                // index into the library's arrays, whose rows may be padded
                ucell.push_back(rc[i].cell / G.n2 * G.pitch + rc[i].cell % G.n2);
            }
            uidx.push_back(rc[i].idx);
            ushot.push_back(rc[i].shot);
        }
        uoff.push_back(nrec);
        P->nuniq = (int)ucell.size();
        HIPCHK(sc.get((void**)&P->d_ucell, sizeof(int64_t) * ucell.size()));
        HIPCHK(sc.get((void**)&P->d_uoff, sizeof(int32_t) * uoff.size()));
        HIPCHK(sc.get((void**)&P->d_uidx, sizeof(int32_t) * uidx.size()));
        HIPCHK(sc.get((void**)&P->d_ushot, sizeof(int32_t) * ushot.size()));
        HIPCHK(hipMemcpyAsync(P->d_ucell, ucell.data(), sizeof(int64_t) * ucell.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_uoff, uoff.data(), sizeof(int32_t) * uoff.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_uidx, uidx.data(), sizeof(int32_t) * uidx.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_ushot, ushot.data(), sizeof(int32_t) * ushot.size(), hipMemcpyHostToDevice, s));
    }
    // the host vectors die with this frame: finish the copies first
    HIPCHK(hipStreamSynchronize(s));

    // second launch shape for the launches without accumulator access
    if (!pairs && G.variant_plain > 0 &&
        (G.variant_plain != G.variant || (G.chunk_plain > 0 && G.chunk_plain != P->chunk))) {
        const fdw::Variant w = fdw::variant_shape(G.ndim, G.variant_plain);
        int gsz = 1;
        for (const Group& gr : P->groups) gsz = std::max(gsz, gr.size);
        if (w.tz != 0 && G.n2 % w.vz == 0 && w.max_shots >= gsz) {
            Geo G2 = G;
            G2.variant = G.variant_plain;
            G2.chunk = G.chunk_plain;
            G2.auto_variant = false;
            G2.variant_plain = 0;
            G2.max_group = gsz;
            auto P2 = std::make_shared<Plan>();
            int rc2 = make_plan(G2, acq, false, s, sc, P2.get());
            if (rc2) return rc2;
            bool same = P2->groups.size() == P->groups.size();
            for (size_t i = 0; same && i < P->groups.size(); ++i)
                same = P2->groups[i].g0 == P->groups[i].g0 && P2->groups[i].size == P->groups[i].size;
            if (same) P->plain = P2;
        }
    }
    return FD_OK;
}

fdw::StepArgs base_args(const Geo& G, const Plan& P, const void* c, double dt)
{
    fdw::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = c;
    a.shot_stride = G.ncell_pad;
    a.n0 = G.n0; a.n1 = G.n1; a.n2 = G.n2;
    a.pitch = G.pitch;
    const double* w = weights(2 * G.r);
    for (int j = 0; j < G.r; ++j) a.w[j] = w[j] / (G.dx * G.dx);
    a.dt2 = dt * dt;
    a.inv_vol = G.inv_vol;
    a.active = 1;
    a.nty = P.nty; a.ntz = P.ntz; a.chunk_len = P.chunk; a.nblk = P.nblk;
    return a;
}

// One step launch of group `gr` with the launch shape of plan P.
int step_group(const Geo& G, const Plan& P, const Group& gr, fdw::StepArgs a, hipStream_t s)
{
    a.blk_off = gr.d_off;
    a.grp = gr.d_grp;
    a.ev = gr.d_ev;
    a.nty = P.nty;
    a.ntz = P.ntz;
    a.chunk_len = P.chunk;
    a.nblk = P.nblk;
    if (a.stiff)
        HIPCHK(fdw::launch_vd_step(G.ndim, G.dtype, G.acc_dtype, P.variant, P.nblk, a, s));
    else
        HIPCHK(fdw::launch_step(G.ndim, G.r, G.dtype, G.acc_dtype, P.variant, gr.size, P.nblk, a, s));
    return FD_OK;
}

// One step launch of shot group gi: launches that touch no accumulator take the plan's
// second launch shape when it has one.
int step(const Geo& G, const Plan& P, int gi, const fdw::StepArgs& a, hipStream_t s)
{
    const bool plain = a.acc_sign == 0 && a.acc_face == 0 && P.plain;
    const Plan& Q = plain ? *P.plain : P;
    return step_group(G, Q, Q.groups[gi], a, s);
}

// Kernel terms of launch l in a run of `count` consecutive accumulating launches of one
// sweep (the interval each completes follows the previous launch's): launch l can add
// its own interval and the one before, so launches 1, 3, 5, ... add pairs and, for odd
// counts, the last one adds its own alone.  The accumulator is then read and written
// by every other launch only.  Returns 0 (none), 1 (own interval) or 3 (both).
int acc_terms(int l, int count)
{
    if (l < 0 || l >= count) return 0;
    if (l & 1) return 3;
    return l == count - 1 ? 1 : 0;
}

void set_acc(fdw::StepArgs& a, int terms, int sign)
{
    a.acc_sign = terms ? sign : 0;
    a.acc_prev = terms == 3;
}

// What accumulating launch l of a run of `count` does with its terms when a partial
// sum buffer is in use: the accumulating launches are numbered i = l / 2 in sweep
// order; each cycle of kPartialCycle of them starts the partial sum, adds to it and
// folds it into the accumulator at its end, and the sweep's last accumulating launch
// folds whatever is pending (or adds directly when nothing is).
int cycle_mode(int i, int total)
{
    const int j = i % fdw::kPartialCycle;
    if (i == total - 1) return j == 0 ? fdw::PM_DIRECT : fdw::PM_FLUSH;
    if (j == 0) return fdw::PM_START;
    return j == fdw::kPartialCycle - 1 ? fdw::PM_FLUSH : fdw::PM_ADD;
}

int part_mode(int l, int count)
{
    return cycle_mode(l >> 1, (count + 1) >> 1);   // the run's accumulating launches
}

bool use_partials(const Geo& G) { return G.dtype == FD_F32 && G.acc_dtype == FD_F64 && !G.no_partials; }

int partial_buffer(const Geo& G, Scratch& sc, void** part)
{
    *part = nullptr;
    if (use_partials(G)) HIPCHK(sc.get(part, G.ncell_pad * sizeof(float)));
    return FD_OK;
}

void set_acc_at(fdw::StepArgs& a, int l, int count, int sign)
{
    const int terms = acc_terms(l, count);
    set_acc(a, terms, sign);
    a.part_mode = (terms && a.part) ? part_mode(l, count) : fdw::PM_DIRECT;
}

void set_face_at(fdw::StepArgs& a, int l, int nlaunch)
{
    a.part_b_mode = (a.acc_face && a.part_b) ? cycle_mode(l, nlaunch) : fdw::PM_DIRECT;
}

int check_time(double dt, int nt)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FD_E_ARG, "dt must be positive and finite");
    if (nt < 1) return fail(FD_E_ARG, "nt must be >= 1");
    return FD_OK;
}

// ---------------------------------------------------------------------------
// two steps per launch
// ---------------------------------------------------------------------------

bool use_pairs(const Geo& G, const fd_acq* acq)
{
    if (G.pairs <= 0 || G.ndim != 3 || (acq && nshots(acq) != 1)) return false;
    return G.n0 >= 2 * G.r && G.n1 >= 2 * G.r && G.n2 >= 2 * G.r;
}

namespace {

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Positions along one axis (in [-r, n + r)) that stand for cell c: the cell itself and
// its mirror images past the walls.
int mirror_positions(int c, int n, int r, int* pos)
{
    int k = 0;
    pos[k++] = c;
    if (-1 - c >= -r) pos[k++] = -1 - c;
    if (2 * n - 1 - c < n + r) pos[k++] = 2 * n - 1 - c;
    return k;
}

}  // namespace

int make_pair_sweep(const Geo& G, const fd_acq* acq, hipStream_t s, Scratch& sc, PairPlan* PP, PairSweep* ws)
{
    constexpr int TZ = fdw::kPairTZ, TY = fdw::kPairTY;
    const int R = G.r;
    Geo T = G;
    T.variant = 1;   // the pair kernel's tile: 64 x 8, one cell per lane
    T.auto_variant = false;
    T.max_group = 1;
    T.variant_plain = 0;
    T.chunk = 0;   // the library's split of axis 0 (chunks of at least 16 r planes in 3D:
                   // the ring adds 2r planes of level n+1 and 2r of queue per chunk)
    int rc = make_plan(T, acq, false, s, sc, &PP->tile);
    if (rc) return rc;
    const Plan& P = PP->tile;
    const int nty = P.nty, ntz = P.ntz, nch = P.nch, C = P.chunk;
    const int nstrip = 2 * R * TZ;
    // ring events: every position of every block's ring of level n+1 that stands for an
    // event's cell, with the plane and lane the kernel walks
    struct Item { int64_t key; fdw::Event e; };
    std::vector<Item> items;
    auto add_cell = [&](int64_t cell, int kind, int idx) {
        const int64_t plane = (int64_t)G.n1 * G.n2;
        const int cx = (int)(cell / plane);
        const int64_t rem = cell - (int64_t)cx * plane;
        const int cy = (int)(rem / G.n2), cz = (int)(rem - (int64_t)cy * G.n2);
        int px[3], py[3], pz[3];
        const int nx = mirror_positions(cx, G.n0, R, px);
        const int ny = mirror_positions(cy, G.n1, R, py);
        const int nz = mirror_positions(cz, G.n2, R, pz);
        for (int ix = 0; ix < nx; ++ix)
            for (int iy = 0; iy < ny; ++iy)
                for (int iz = 0; iz < nz; ++iz) {
                    const int x = px[ix], y = py[iy], z = pz[iz];
                    auto emit = [&](int tyb, int tzb, int lane) {
                        for (int ch = floordiv(x, C) - 1; ch <= floordiv(x, C) + 1; ++ch) {
                            if (ch < 0 || ch >= nch) continue;
                            const int x0 = ch * C, x1 = std::min(x0 + C, G.n0);
                            if (x < x0 - R || x >= x1 + R) continue;
                            fdw::Event e;
                            e.plane = x;
                            e.lane = lane;
                            e.kind = kind;
                            e.idx = idx;
                            items.push_back({((int64_t)ch * nty + tyb) * ntz + tzb, e});
                        }
                    };
                    const bool yin = y >= 0 && y < nty * TY, zin = z >= 0 && z < ntz * TZ;
                    if (yin && zin) {   // a tile cell
                        const int tyb = y / TY, tzb = z / TZ;
                        emit(tyb, tzb, (y - tyb * TY) * TZ + (z - tzb * TZ));
                    }
                    if (zin) {          // ring rows above and below tiles
                        const int tzb = z / TZ;
                        for (int tyb = floordiv(y, TY) - 1; tyb <= floordiv(y, TY) + 1; ++tyb) {
                            if (tyb < 0 || tyb >= nty) continue;
                            const int y0 = tyb * TY;
                            int sr = -1;
                            if (y >= y0 - R && y < y0) sr = y - (y0 - R);
                            else if (y >= y0 + TY && y < y0 + TY + R) sr = R + (y - (y0 + TY));
                            if (sr >= 0) emit(tyb, tzb, TY * TZ + sr * TZ + (z - tzb * TZ));
                        }
                    }
                    if (yin) {          // ring columns left and right of tiles
                        const int tyb = y / TY;
                        for (int tzb = floordiv(z, TZ) - 1; tzb <= floordiv(z, TZ) + 1; ++tzb) {
                            if (tzb < 0 || tzb >= ntz) continue;
                            const int z0 = tzb * TZ;
                            int side = -1, col = 0;
                            if (z >= z0 - R && z < z0) { side = 0; col = z - (z0 - R); }
                            else if (z >= z0 + TZ && z < z0 + TZ + R) { side = 1; col = z - (z0 + TZ); }
                            if (side >= 0)
                                emit(tyb, tzb, TY * TZ + nstrip + side * (R * TY) + (y - tyb * TY) * R + col);
                        }
                    }
                }
    };
    const int nsrc = acq ? acq->nsrc : 0;
    const int nrec = acq ? acq->nrec : 0;
    for (int i = 0; i < nsrc; ++i) add_cell(acq->src_cell[i], fdw::EV_SRC, i);
    for (int i = 0; i < nrec; ++i) add_cell(acq->rec_cell[i], fdw::EV_REC, i);
    std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.e.plane != b.e.plane) return a.e.plane < b.e.plane;
        if (a.e.lane != b.e.lane) return a.e.lane < b.e.lane;
        if (a.e.kind != b.e.kind) return a.e.kind < b.e.kind;
        return a.e.idx < b.e.idx;
    });
    std::vector<int32_t> off(P.nblk + 1, 0);
    std::vector<fdw::EvPlane> grp;
    std::vector<fdw::Event> ev(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        ev[i] = items[i].e;
        if (i == 0 || items[i].key != items[i - 1].key || ev[i].plane != ev[i - 1].plane) {
            fdw::EvPlane g;
            g.plane = ev[i].plane;
            g.begin = g.end = (int32_t)i;
            g.pad = 0;
            grp.push_back(g);
            off[items[i].key + 1]++;
        }
        grp.back().end = (int32_t)i + 1;
    }
    for (int b = 0; b < P.nblk; ++b) off[b + 1] += off[b];
    // every block's groups lie on planes its walk visits, in increasing order, with
    // ranges inside the event table (the kernel reads the table where these say)
    for (int b = 0; b < P.nblk; ++b) {
        const int ch = b / (ntz * nty);
        const int x0 = ch * C, x1 = std::min(x0 + C, G.n0);
        for (int g = off[b]; g < off[b + 1]; ++g) {
            const fdw::EvPlane& q = grp[g];
            if (q.plane < x0 - R || q.plane >= x1 + R || (g > off[b] && q.plane <= grp[g - 1].plane) ||
                q.begin < 0 || q.end <= q.begin || q.end > (int32_t)ev.size())
                return fail(FD_E_DEVICE, "internal error: inconsistent ring event table");
        }
    }
    HIPCHK(sc.get((void**)&PP->d_off_a, sizeof(int32_t) * off.size()));
    HIPCHK(sc.get((void**)&PP->d_grp_a, sizeof(fdw::EvPlane) * std::max<size_t>(1, grp.size())));
    HIPCHK(sc.get((void**)&PP->d_ev_a, sizeof(fdw::Event) * std::max<size_t>(1, ev.size())));
    HIPCHK(hipMemcpyAsync(PP->d_off_a, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, s));
    if (!grp.empty())
        HIPCHK(hipMemcpyAsync(PP->d_grp_a, grp.data(), sizeof(fdw::EvPlane) * grp.size(), hipMemcpyHostToDevice, s));
    if (!ev.empty())
        HIPCHK(hipMemcpyAsync(PP->d_ev_a, ev.data(), sizeof(fdw::Event) * ev.size(), hipMemcpyHostToDevice, s));
    if (ws) {
        ws->pp = PP;
        const size_t fb = G.ncell_pad * dsize(G.dtype);
        HIPCHK(sc.get(&ws->xa, fb));
        HIPCHK(sc.get(&ws->xb, fb));
    }
    HIPCHK(hipStreamSynchronize(s));   // the host tables die with this frame
    return FD_OK;
}

namespace {

// Kernel terms of the two-step launch over steps l, l + 1 of a run of `count`
// accumulating steps: both intervals when step l + 1 adds two in the one-step schedule,
// the first alone when step l is the run's last accumulating step; the partial-sum
// mode of that step.
void set_pair_acc(fdw::PairArgs& p, int l, int count, int sign)
{
    const int ta = acc_terms(l, count), tb = acc_terms(l + 1, count);
    int terms = 0, at = 0;
    if (tb == 3) { terms = 3; at = l + 1; }
    else if (ta != 0) { terms = 1; at = l; }
    p.terms = terms;
    p.s.acc_sign = terms ? sign : 0;
    p.s.acc_prev = 0;
    p.s.part_mode = (terms && p.s.part) ? part_mode(at, count) : fdw::PM_DIRECT;
}

fdw::PairArgs pair_args(const Geo& G, const PairPlan& PP, const void* c, double dt, const fd_acq* acq)
{
    fdw::PairArgs p;
    std::memset(&p, 0, sizeof(p));
    p.s = base_args(G, PP.tile, c, dt);
    p.s.blk_off = PP.tile.groups[0].d_off;
    p.s.grp = PP.tile.groups[0].d_grp;
    p.s.ev = PP.tile.groups[0].d_ev;
    p.s.wavelet = acq->wavelet;
    p.s.nsrc = acq->nsrc;
    p.s.nrec = acq->nrec;
    p.blk_off_a = PP.d_off_a;
    p.grp_a = PP.d_grp_a;
    p.ev_a = PP.d_ev_a;
    return p;
}

}  // namespace

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
        if ((rc = check_speeds({G}, {c}, {dt}, s, sc))) return rc;
    }
    return FD_OK;
}

// Forward sweep of every shot group (Alg. 1 forward loop); the wavefields of shot s
// live at ua/ub + s * ncell_pad (rows possibly padded to G.pitch).  `acc` null: no kernel accumulation (plain forward).  With
// vd.stiff the variable-material step runs (c is then the mass coefficient) and, with
// vd.acc_b, every launch adds the stiffness term of its current level (through the
// partial sums vd.part_b when given).
int forward_sweep(const Geo& G, const Plan& P, const void* c, const fd_acq* acq, double dt, int nt,
                  const void* obs, void* ua, void* ub, void* acc, void* resid, void* traces,
                  hipStream_t s, const VdFields& vd, void* part, const PairSweep* pw)
{
    const size_t fb = G.ncell_pad * dsize(G.dtype) * nshots(acq);
    HIPCHK(hipMemsetAsync(ua, 0, fb, s));
    HIPCHK(hipMemsetAsync(ub, 0, fb, s));
    if (acc) HIPCHK(hipMemsetAsync(acc, 0, G.ncell_pad * dsize(G.acc_dtype), s));
    if (vd.acc_b) HIPCHK(hipMemsetAsync(vd.acc_b, 0, G.ncell_pad * dsize(G.acc_dtype), s));
    fdw::StepArgs a = base_args(G, P, c, dt);
    a.acc = acc;
    a.part = part;
    a.stiff = vd.stiff;
    a.acc_b = vd.acc_b;
    a.part_b = vd.acc_b ? vd.part_b : nullptr;
    a.acc_face = vd.acc_b ? 1 : 0;   // levels 0..nt-1 (level 0 is zero)
    a.wavelet = acq->wavelet;
    a.nsrc = acq->nsrc;
    a.sample = 1;
    a.traces = traces;
    a.resid = resid;
    a.obs = obs;
    a.nrec = acq->nrec;
    const size_t es = dsize(G.dtype);
    SweepTimer tm(G.timing != nullptr, s);
    tm.start();
    int pair_launches = 0;
    if (pw && pw->pp && !vd.stiff) {
        // two steps per launch, alternating between the pairs (ua, ub) and (xa, xb); a
        // last odd step runs as one step in place
        fdw::PairArgs p = pair_args(G, *pw->pp, c, dt, acq);
        p.s.acc = acc;
        p.s.part = part;
        p.s.sample = 1;
        p.s.traces = traces;
        p.s.resid = resid;
        p.s.obs = obs;
        void* bufs[2][2] = {{ua, ub}, {pw->xa, pw->xb}};
        int k = 0, n = 0;
        for (; n + 1 < nt; n += 2, k ^= 1) {
            p.s.unew = bufs[k][0];
            p.s.ucur = bufs[k][1];
            p.out1 = bufs[k ^ 1][0];
            p.out2 = bufs[k ^ 1][1];
            p.s.row_src = p.s.row_rec = n;
            p.row_src2 = p.row_rec2 = n + 1;
            if (acc) set_pair_acc(p, n, nt - 1, 1);
            else p.terms = 0;
            HIPCHK(fdw::launch_pair(G.r, G.dtype, G.acc_dtype, pw->pp->tile.nblk, p, s));
            ++pair_launches;
        }
        void* prev = bufs[k][0];
        void* cur = bufs[k][1];
        if (n < nt) {
            a.ucur = cur;
            a.unew = prev;
            if (acc) set_acc_at(a, n, nt - 1, 1);
            else set_acc(a, 0, 1);
            a.row_src = a.row_rec = n;
            int rc = step(G, P, 0, a, s);
            if (rc) return rc;
        }
        // after an odd number of two-step launches the levels sit in (xa, xb): move them
        // to where final_levels names them
        if (k == 1) {
            HIPCHK(hipMemcpyAsync(ua, pw->xa, G.ncell_pad * es, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(ub, pw->xb, G.ncell_pad * es, hipMemcpyDeviceToDevice, s));
        }
        tm.stop();
        if (G.timing) {
            G.timing->fwd_ms = tm.ms();
            G.timing->fwd_launches = pair_launches + (nt & 1);
            G.timing->fwd_pair_launches = pair_launches;
            G.timing->persistent_blocks = 0;
        }
        return FD_OK;
    }
    for (int gi = 0; gi < (int)P.groups.size(); ++gi) {
        const Group& gr = P.groups[gi];
        char* prev = (char*)ua + (size_t)gr.g0 * G.ncell_pad * es;   // level n-1
        char* cur = (char*)ub + (size_t)gr.g0 * G.ncell_pad * es;    // level n
        for (int n = 0; n < nt; ++n) {
            a.ucur = cur;
            a.unew = prev;
            // intervals 0..nt-2; the last one is settled at hand-over
            if (acc) set_acc_at(a, n, nt - 1, 1);
            else set_acc(a, 0, 1);
            set_face_at(a, n, nt);
            a.row_src = n;
            a.row_rec = n;
            int rc = step(G, P, gi, a, s);
            if (rc) return rc;
            std::swap(prev, cur);
        }
    }
    tm.stop();
    if (G.timing) {
        G.timing->fwd_ms = tm.ms();
        G.timing->fwd_launches = nt * (int)P.groups.size();
        G.timing->fwd_pair_launches = 0;
        G.timing->persistent_blocks = 0;
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
                   double k, void* ua, void* ub, void* acc, void* resid, hipStream_t s,
                   const VdFields& vd, void* part, const PairSweep* pw)
{
    void* up = nullptr;   // u^{nt-1} -> v^{nt-1}
    void* ul = nullptr;   // u^nt = v^nt
    final_levels(ua, ub, nt, &up, &ul);
    const double rec_scale = -k / dt;   // k fdag^n = -(k/dt) residual^n
    const size_t es = dsize(G.dtype);
    fdw::StepArgs a = base_args(G, P, c, dt);
    a.acc = acc;
    a.part = part;
    a.stiff = vd.stiff;
    a.acc_b = vd.acc_b;
    a.part_b = vd.acc_b ? vd.part_b : nullptr;
    a.acc_face = vd.acc_b ? -1 : 0;   // levels nt-1..1 of the superposed field
    a.wavelet = acq->wavelet;
    a.nsrc = acq->nsrc;
    a.inject_rec = 1;
    a.resid = resid;
    a.nrec = acq->nrec;
    a.rec_scale = rec_scale;
    SweepTimer tm(G.timing != nullptr && nt > 1, s);
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const Group& gr = P.groups[gi];
        char* vj = (char*)up + (size_t)gr.g0 * G.ncell_pad * es;   // v^j
        char* vn = (char*)ul + (size_t)gr.g0 * G.ncell_pad * es;   // v^{j+1}, overwritten by v^{j-1}
        if (acq->nrec > 0)
            HIPCHK(fdw::launch_terminal(G.dtype, G.acc_dtype, P.nuniq, P.d_ucell, P.d_uoff, P.d_uidx,
                                        P.d_ushot, gr.g0, gr.size, G.ncell_pad, c, vd.stiff ? 1 : 0,
                                        dt * dt, vn, vj, acc,
                                        (const char*)resid + (size_t)(nt - 1) * acq->nrec * es,
                                        rec_scale, s));
        if (gi == 0) tm.start();
        if (pw && pw->pp && !vd.stiff) {
            // steps j, j - 1 per launch (l = nt - 1 - j even), a last odd step in place
            fdw::PairArgs p = pair_args(G, *pw->pp, c, dt, acq);
            p.s.acc = acc;
            p.s.part = part;
            p.s.inject_rec = 1;
            p.s.resid = resid;
            p.s.rec_scale = rec_scale;
            void* bufs[2][2] = {{vn, vj}, {pw->xa, pw->xb}};   // (level j+1, level j)
            int kk = 0, l = 0, pairs = 0;
            for (; l + 1 < nt - 1; l += 2, kk ^= 1) {
                const int j = nt - 1 - l;
                p.s.unew = bufs[kk][0];
                p.s.ucur = bufs[kk][1];
                p.out1 = bufs[kk ^ 1][0];
                p.out2 = bufs[kk ^ 1][1];
                p.s.row_src = j;
                p.s.row_rec = j - 1;
                p.row_src2 = j - 1;
                p.row_rec2 = j - 2;
                set_pair_acc(p, l, nt - 1, -1);
                HIPCHK(fdw::launch_pair(G.r, G.dtype, G.acc_dtype, pw->pp->tile.nblk, p, s));
                ++pairs;
            }
            if (l < nt - 1) {
                const int j = nt - 1 - l;
                a.ucur = bufs[kk][1];
                a.unew = bufs[kk][0];
                a.row_src = j;
                a.row_rec = j - 1;
                set_acc_at(a, l, nt - 1, -1);
                int rc = step(G, P, (int)gi, a, s);
                if (rc) return rc;
            }
            tm.stop();
            if (G.timing) {
                G.timing->bwd_ms = tm.ms();
                G.timing->bwd_launches = pairs + ((nt - 1) & 1);
                G.timing->bwd_pair_launches = pairs;
            }
            return FD_OK;
        }
        for (int j = nt - 1; j >= 1; --j) {
            a.ucur = vj;
            a.unew = vn;
            a.row_src = j;
            a.row_rec = j - 1;
            set_acc_at(a, nt - 1 - j, nt - 1, -1);   // intervals nt-2..0
            set_face_at(a, nt - 1 - j, nt - 1);
            int rc = step(G, P, (int)gi, a, s);
            if (rc) return rc;
            std::swap(vj, vn);
        }
    }
    tm.stop();
    if (G.timing) {
        G.timing->bwd_ms = tm.ms();
        G.timing->bwd_launches = (nt - 1) * (int)P.groups.size();
        G.timing->bwd_pair_launches = 0;
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

// Rows that do not start on 256-byte boundaries cost about a third of a sweep's
// throughput (each 64-lane row load touches three cache lines instead of two): the
// sweeps of the calls that use this run on copies whose rows are padded to 64
// elements.  The caller's arrays stay dense.
void pad_rows(Geo* G)
{
    const int pitch = (G->n2 + 63) / 64 * 64;
    if (pitch != G->n2 && (int64_t)G->n1 * pitch < ((int64_t)1 << 31)) {
        G->pitch = pitch;
        G->ncell_pad = (int64_t)G->n0 * G->n1 * pitch;
    }
}

// Copy `rows` rows of n2 elements between arrays with row strides dpitch and spitch.
int copy_rows(void* dst, int64_t dpitch, const void* src, int64_t spitch, size_t es, int64_t rows, int64_t n2,
              hipStream_t s)
{
    if (rows == 0) return FD_OK;
    HIPCHK(fdw::launch_copy_rows(dst, dpitch, src, spitch, es, rows, n2, s));
    return FD_OK;
}

// One field in the library's row layout: the caller's array when rows are not padded,
// else a padded copy.
int padded_field(const Geo& G, const void* f, Scratch& sc, hipStream_t s, const void** fp)
{
    *fp = f;
    if (G.pitch == G.n2) return FD_OK;
    const size_t es = dsize(G.dtype);
    void* p = nullptr;
    HIPCHK(sc.get(&p, G.ncell_pad * es));
    int rc = copy_rows(p, G.pitch, f, G.n2, es, (int64_t)G.n0 * G.n1, G.n2, s);
    if (rc) return rc;
    *fp = p;
    return FD_OK;
}

// The material of a sweep in the library's row layout: the caller's arrays when rows
// are not padded, else padded copies.
int padded_material(const Geo& G, const void* m, const void* b, Scratch& sc, hipStream_t s, const void** mp,
                    const void** bp)
{
    *mp = m;
    *bp = b;
    if (G.pitch == G.n2) return FD_OK;
    const size_t es = dsize(G.dtype);
    const int64_t rows = (int64_t)G.n0 * G.n1;
    void *pm = nullptr, *pb = nullptr;
    HIPCHK(sc.get(&pm, G.ncell_pad * es));
    HIPCHK(sc.get(&pb, G.ncell_pad * es));
    int rc;
    if ((rc = copy_rows(pm, G.pitch, m, G.n2, es, rows, G.n2, s))) return rc;
    if ((rc = copy_rows(pb, G.pitch, b, G.n2, es, rows, G.n2, s))) return rc;
    *mp = pm;
    *bp = pb;
    return FD_OK;
}

int vd_work(const Geo& G, const fd_state* st, void* acc_b, int ns, bool own_state, bool copy_in, Scratch& sc,
            hipStream_t s, VdWork* w)
{
    w->st = *st;
    w->acc_b = acc_b;
    if (G.pitch == G.n2 || own_state) return FD_OK;
    const size_t es = dsize(G.dtype), aes = dsize(G.acc_dtype);
    HIPCHK(sc.get(&w->st.u_a, G.ncell_pad * es * ns));
    HIPCHK(sc.get(&w->st.u_b, G.ncell_pad * es * ns));
    HIPCHK(sc.get(&w->st.acc, G.ncell_pad * aes));
    if (acc_b) HIPCHK(sc.get(&w->acc_b, G.ncell_pad * aes));
    w->copied = true;
    if (!copy_in) return FD_OK;
    const int64_t rows = (int64_t)G.n0 * G.n1;
    int rc;
    if ((rc = copy_rows(w->st.u_a, G.pitch, st->u_a, G.n2, es, rows * ns, G.n2, s))) return rc;
    if ((rc = copy_rows(w->st.u_b, G.pitch, st->u_b, G.n2, es, rows * ns, G.n2, s))) return rc;
    if ((rc = copy_rows(w->st.acc, G.pitch, st->acc, G.n2, aes, rows, G.n2, s))) return rc;
    return acc_b ? copy_rows(w->acc_b, G.pitch, acc_b, G.n2, aes, rows, G.n2, s) : FD_OK;
}

// Hand a padded working state back to the caller's dense arrays.
int work_out(const Geo& G, const VdWork& w, const fd_state* st, void* acc_b, int ns, hipStream_t s)
{
    if (!w.copied) return FD_OK;
    const size_t es = dsize(G.dtype), aes = dsize(G.acc_dtype);
    const int64_t rows = (int64_t)G.n0 * G.n1;
    int rc;
    if ((rc = copy_rows(st->u_a, G.n2, w.st.u_a, G.pitch, es, rows * ns, G.n2, s))) return rc;
    if ((rc = copy_rows(st->u_b, G.n2, w.st.u_b, G.pitch, es, rows * ns, G.n2, s))) return rc;
    if ((rc = copy_rows(st->acc, G.n2, w.st.acc, G.pitch, aes, rows, G.n2, s))) return rc;
    return acc_b ? copy_rows(acc_b, G.n2, w.acc_b, G.pitch, aes, rows, G.n2, s) : FD_OK;
}

int check_state(const fd_state* st, const Geo& G, int nt, const fd_acq* acq)
{
    if (!st) return fail(FD_E_ARG, "state is null");
    const size_t fb = G.ncell * dsize(G.dtype) * nshots(acq);
    int rc;
    if ((rc = check_dev(st->u_a, fb, "state.u_a"))) return rc;
    if ((rc = check_dev(st->u_b, fb, "state.u_b"))) return rc;
    if ((rc = check_dev(st->acc, G.ncell * dsize(G.acc_dtype), "state.acc"))) return rc;
    if ((rc = check_dev(st->residual, (size_t)nt * acq->nrec * dsize(G.dtype), "state.residual"))) return rc;
    return FD_OK;
}

}  // namespace fdh
