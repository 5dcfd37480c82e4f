// fdwave C-ABI: argument validation, CFL check, block plans, device scratch and the
// time loops of the paper's Algorithm 1 (forward sweep, terminal hand-over,
// superposed backward sweep, finalisation), for one problem with one or more shots
// and for batches of independent problems.  Kernels live in fdw_step.hip and
// fdw_kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdwave.h"
#include "fdw_aux.h"
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
    int max_group = 0;   // requested shots per launch (0: the variant's largest)
    int graph = 0;
    int persistent = 0;
    int barrier_timeout_us = 0;
    bool auto_variant = true;   // the caller left the variant to the library
    int variant_plain = 0;      // launches without accumulator access: tile variant (0: variant)
    int chunk_plain = 0;        //   and planes per block (0: library choice)
    int n0, n1, n2;      // internal extents (2D: n1 = 1)
    int64_t ncell;
    int pitch = 0;       // row stride of the library's own arrays (>= n2; see vd_setup)
    int64_t ncell_pad = 0;   // n0 * n1 * pitch: elements of one such array
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

// One shot group of a plan: shots [g0, g0 + size) and their events: per block a range
// of plane groups (d_off), each a range of events (d_grp), sorted by plane.
struct Group {
    int g0 = 0, size = 1;
    int32_t* d_off = nullptr;
    fdw::EvPlane* d_grp = nullptr;
    fdw::Event* d_ev = nullptr;
};

// Block decomposition, shot groups with their per-block event lists, and the distinct
// receiver cells (terminal hand-over).
struct Plan {
    fdw::Variant v;
    int variant = 1;
    int nty = 0, ntz = 0, nch = 0, chunk = 0, nblk = 0;
    // the launch shape of the launches that do not touch the accumulator, when it
    // differs and groups the shots the same way (else null: this plan serves both)
    std::shared_ptr<Plan> plain;
    std::vector<Group> groups;
    int nuniq = 0;
    int64_t* d_ucell = nullptr;
    int32_t* d_uoff = nullptr;
    int32_t* d_uidx = nullptr;
    int32_t* d_ushot = nullptr;
};

bool apply_tuned(Geo& G, int nshot);

// `pairs`: one group per shot carrying two fields, the shot's wavefield in slot 0 (its
// sources inject there) and its adjoint field in slot 1 (its receivers inject there).
int make_plan(Geo& G, const fd_acq* acq, bool want_uniq, hipStream_t s, Scratch& sc, Plan* P,
              bool pairs = false)
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

// The variable-material fields of a sweep: stiffness b and its accumulator (null for
// the constant-density scheme, whose c argument is then the speed, not the mass).
struct VdFields {
    const void* stiff = nullptr;
    void* acc_b = nullptr;
};

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
        if ((rc = check_speeds({G}, {c}, {dt}, s, sc))) return rc;
    }
    return FD_OK;
}

// Forward sweep of every shot group (Alg. 1 forward loop); the wavefields of shot s
// live at ua/ub + s * ncell_pad (rows possibly padded to G.pitch).  `acc` null: no kernel accumulation (plain forward).  With
// vd.stiff the variable-material step runs (c is then the mass coefficient) and, with
// vd.acc_b, every launch adds the stiffness term of its current level.
int forward_sweep(const Geo& G, const Plan& P, const void* c, const fd_acq* acq, double dt, int nt,
                  const void* obs, void* ua, void* ub, void* acc, void* resid, void* traces,
                  hipStream_t s, const VdFields& vd = VdFields())
{
    const size_t fb = G.ncell_pad * dsize(G.dtype) * nshots(acq);
    HIPCHK(hipMemsetAsync(ua, 0, fb, s));
    HIPCHK(hipMemsetAsync(ub, 0, fb, s));
    if (acc) HIPCHK(hipMemsetAsync(acc, 0, G.ncell_pad * dsize(G.acc_dtype), s));
    if (vd.acc_b) HIPCHK(hipMemsetAsync(vd.acc_b, 0, G.ncell_pad * dsize(G.acc_dtype), s));
    fdw::StepArgs a = base_args(G, P, c, dt);
    a.acc = acc;
    a.stiff = vd.stiff;
    a.acc_b = vd.acc_b;
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
    for (int gi = 0; gi < (int)P.groups.size(); ++gi) {
        const Group& gr = P.groups[gi];
        char* prev = (char*)ua + (size_t)gr.g0 * G.ncell_pad * es;   // level n-1
        char* cur = (char*)ub + (size_t)gr.g0 * G.ncell_pad * es;    // level n
        for (int n = 0; n < nt; ++n) {
            a.ucur = cur;
            a.unew = prev;
            // intervals 0..nt-2; the last one is settled at hand-over
            set_acc(a, acc ? acc_terms(n, nt - 1) : 0, 1);
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
                   const VdFields& vd = VdFields())
{
    void* up = nullptr;   // u^{nt-1} -> v^{nt-1}
    void* ul = nullptr;   // u^nt = v^nt
    final_levels(ua, ub, nt, &up, &ul);
    const double rec_scale = -k / dt;   // k fdag^n = -(k/dt) residual^n
    const size_t es = dsize(G.dtype);
    fdw::StepArgs a = base_args(G, P, c, dt);
    a.acc = acc;
    a.stiff = vd.stiff;
    a.acc_b = vd.acc_b;
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
        for (int j = nt - 1; j >= 1; --j) {
            a.ucur = vj;
            a.unew = vn;
            a.row_src = j;
            a.row_rec = j - 1;
            set_acc(a, acc_terms(nt - 1 - j, nt - 1), -1);   // intervals nt-2..0
            int rc = step(G, P, (int)gi, a, s);
            if (rc) return rc;
            std::swap(vj, vn);
        }
    }
    tm.stop();
    if (G.timing) {
        G.timing->bwd_ms = tm.ms();
        G.timing->bwd_launches = (nt - 1) * (int)P.groups.size();
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
    HIPCHK(hipMemcpy2DAsync(dst, (size_t)dpitch * es, src, (size_t)spitch * es, (size_t)n2 * es, (size_t)rows,
                            hipMemcpyDeviceToDevice, s));
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

// The sweep state in the library's row layout (stiffness accumulator only for the
// variable-material scheme).  With padded rows and a caller-owned
// (dense) state, the sweeps work on padded copies: the forward half hands the final
// levels and both accumulators back to the caller's arrays, the backward half starts
// by copying them in.  Internal states (own_state) are allocated padded.
struct VdWork {
    fd_state st{};
    void* acc_b = nullptr;
    bool copied = false;
};

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

// `own_state`: the state arrays were allocated by the library itself in this call.
int sens_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
                 const void* observed, const fd_state* st, void* traces, double* J_host,
                 const fd_opts* opts, hipStream_t s, bool own_state)
{
    Scratch sc(s);
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, true);
    if (rc) return rc;
    if (!own_state && (rc = check_state(st, G, nt, acq))) return rc;
    const size_t tb = (size_t)nt * acq->nrec * dsize(G.dtype);
    if ((rc = check_dev(observed, tb, "observed"))) return rc;
    if (traces && (rc = check_dev(traces, tb, "traces"))) return rc;
    pad_rows(&G);
    const void* cp = nullptr;
    if ((rc = padded_field(G, c, sc, s, &cp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, false, s, sc, &P))) return rc;
    const int ns = nshots(acq);
    VdWork w;
    if ((rc = vd_work(G, st, nullptr, ns, own_state, false, sc, s, &w))) return rc;
    if ((rc = forward_sweep(G, P, cp, acq, dt, nt, observed, w.st.u_a, w.st.u_b, w.st.acc, st->residual,
                            traces, s)))
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
                  bool own_state)
{
    Scratch sc(s);
    Geo G;
    int rc = prepare(grid, c, acq, dt, nt, opts, s, sc, &G, false);
    if (rc) return rc;
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    if (!std::isfinite(grad_scale)) return fail(FD_E_ARG, "grad_scale must be finite");
    if (!own_state && (rc = check_state(st, G, nt, acq))) return rc;
    if ((rc = check_dev(grad, G.ncell * dsize(G.dtype), "grad_c"))) return rc;
    pad_rows(&G);
    const void* cp = nullptr;
    if ((rc = padded_field(G, c, sc, s, &cp))) return rc;
    Plan P;
    if ((rc = make_plan(G, acq, true, s, sc, &P))) return rc;
    VdWork w;
    if ((rc = vd_work(G, st, nullptr, nshots(acq), own_state, true, sc, s, &w))) return rc;
    if ((rc = backward_sweep(G, P, cp, acq, dt, nt, k, w.st.u_a, w.st.u_b, w.st.acc, st->residual, s)))
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
        G->variant = 1;   // one cell per lane: fits every extent and measured fastest
        G->auto_variant = false;
    } else if (G->variant != 1 && G->variant != 2 &&
               !(G->ndim == 2 && (G->variant == 4 || G->variant == 5))) {
        return fail(FD_E_ARG, "the variable-material scheme runs tile variants 1 and 2 (2D also 4 and 5)");
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
    if ((rc = forward_sweep(G, P, mp, acq, dt, nt, observed, w.st.u_a, w.st.u_b, w.st.acc, st->residual, traces,
                            s, vd)))
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
    if ((rc = backward_sweep(G, P, mp, acq, dt, nt, k, w.st.u_a, w.st.u_b, w.st.acc, st->residual, s, vd)))
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
            G.variant = (G.n2 % 2 == 0) ? 2 : 1;
            G.chunk = 0;
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
            set_acc(a, acc_terms(nt - 1 - j, nt - 1), 1);   // intervals nt-2..0
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

// ---------------------------------------------------------------------------
// autotuner: remembered launch shapes per (arch, runtime, problem class)
// ---------------------------------------------------------------------------

struct Tuned {
    int variant = 1, chunk = 0, group = 1;
    int variant_plain = 0, chunk_plain = 0;   // launches without accumulator access (0: same)
    double ms = 0.0;
};

std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;
bool g_tune_loaded = false;

std::string device_tag()
{
    int dev = 0, rt = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    (void)hipRuntimeGetVersion(&rt);
    return arch + "|hip" + std::to_string(rt);
}

std::string tune_key(const Geo& G, int nshot)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s|%dd|o%d|%s|acc%s|%dx%dx%d|s%d", device_tag().c_str(), G.ndim,
             2 * G.r, G.dtype == FD_F64 ? "f64" : "f32", G.acc_dtype == FD_F64 ? "f64" : "f32",
             G.n0, G.n1, G.n2, nshot);
    return buf;
}

const char* tune_file() { return std::getenv("FDWAVE_TUNE_CACHE"); }

// Reads "key" and the numbers after "variant", "chunk", "max_group", "variant_plain",
// "chunk_plain" and "ms" from one JSON line written by tune_save (no general JSON parser
// is needed for that format).
bool parse_line(const std::string& ln, std::string* key, Tuned* t)
{
    auto str_after = [&](const char* name, std::string* out) {
        const std::string pat = std::string("\"") + name + "\": \"";
        size_t p = ln.find(pat);
        if (p == std::string::npos) return false;
        p += pat.size();
        size_t q = ln.find('"', p);
        if (q == std::string::npos) return false;
        *out = ln.substr(p, q - p);
        return true;
    };
    auto num_after = [&](const char* name, double* out) {
        const std::string pat = std::string("\"") + name + "\": ";
        size_t p = ln.find(pat);
        if (p == std::string::npos) return false;
        *out = std::atof(ln.c_str() + p + pat.size());
        return true;
    };
    double v, c, g, ms, vp = 0.0, cp = 0.0;
    if (!str_after("key", key) || !num_after("variant", &v) || !num_after("chunk", &c) ||
        !num_after("max_group", &g) || !num_after("ms", &ms))
        return false;
    (void)num_after("variant_plain", &vp);   // absent in entries with one launch shape
    (void)num_after("chunk_plain", &cp);
    t->variant = (int)v;
    t->chunk = (int)c;
    t->group = (int)g;
    t->variant_plain = (int)vp;
    t->chunk_plain = (int)cp;
    t->ms = ms;
    return true;
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = tune_file();
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        std::string key;
        Tuned t;
        if (parse_line(line, &key, &t)) g_tuned[key] = t;   // later lines win
    }
    std::fclose(f);
}

void tune_save_locked(const std::string& key, const Tuned& t)
{
    g_tuned[key] = t;
    const char* path = tune_file();
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"variant\": %d, \"chunk\": %d, \"max_group\": %d, "
                 "\"variant_plain\": %d, \"chunk_plain\": %d, \"ms\": %.6f}\n",
                 key.c_str(), t.variant, t.chunk, t.group, t.variant_plain, t.chunk_plain, t.ms);
    std::fclose(f);
}

// Applies the remembered launch shape of (G, nshot), if any; returns whether there was one.
bool apply_tuned(Geo& G, int nshot)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tuned.find(tune_key(G, nshot));
    if (it == g_tuned.end()) return false;
    const fdw::Variant v = fdw::variant_shape(G.ndim, it->second.variant);
    if (v.tz == 0 || G.n2 % v.vz != 0) return false;
    G.variant = it->second.variant;
    if (G.chunk == 0) G.chunk = it->second.chunk;
    if (G.max_group == 0) G.max_group = it->second.group;
    if (G.variant_plain == 0) {
        G.variant_plain = it->second.variant_plain;
        if (G.chunk_plain == 0) G.chunk_plain = it->second.chunk_plain;
    }
    return true;
}

int autotune(const fd_grid* grid, int nshot, const fd_opts* opts, int steps, fd_opts* best,
             double* best_ms, hipStream_t s)
{
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if (!best) return fail(FD_E_ARG, "best is null");
    if (steps < 1) return fail(FD_E_ARG, "steps must be >= 1");
    // small grids give launches of tens of microseconds: time more of them
    steps *= (int)std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)1 << 26) / std::max<int64_t>(G.ncell, 1)));
    nshot = std::max(nshot, 1);
    // candidate shapes: variants that fit, shot groups, chunk lengths
    std::vector<int> groups = {1};
    if (nshot >= 2) groups.push_back(2);
    if (nshot >= 4) groups.push_back(4);
    int gmax = 1;
    for (int g : groups) gmax = std::max(gmax, g);
    struct Scoped {
        std::vector<void*> p;
        ~Scoped() { for (void* q : p) (void)hipFree(q); }
    } mem;
    const size_t es = dsize(G.dtype);
    void *c = nullptr, *ua = nullptr, *ub = nullptr, *acc = nullptr;
    HIPCHK(hipMalloc(&c, G.ncell * es)); mem.p.push_back(c);
    HIPCHK(hipMalloc(&ua, G.ncell * es * gmax)); mem.p.push_back(ua);
    HIPCHK(hipMalloc(&ub, G.ncell * es * gmax)); mem.p.push_back(ub);
    HIPCHK(hipMalloc(&acc, G.ncell * dsize(G.acc_dtype))); mem.p.push_back(acc);
    HIPCHK(hipMemsetAsync(c, 0, G.ncell * es, s));
    HIPCHK(hipMemsetAsync(ua, 0, G.ncell * es * gmax, s));
    HIPCHK(hipMemsetAsync(ub, 0, G.ncell * es * gmax, s));
    HIPCHK(hipMemsetAsync(acc, 0, G.ncell * dsize(G.acc_dtype), s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct Ev { hipEvent_t a, b; ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evs{e0, e1};
    // per shot-group size: the fastest shape of the launches that add kernel terms and,
    // separately, of the launches that touch no accumulator (the sweeps alternate them)
    struct Best { double ms = 1e300; int variant = 0, chunk = 0; };
    std::map<int, Best> best_acc, best_plain, best_same;
    auto time_launches = [&](const Geo& T, const Plan& P, const Group& gr, fdw::StepArgs a, int terms,
                             double* ms_out) -> int {
        void *prev = ua, *cur = ub;
        for (int n = 0; n < steps + 1; ++n) {   // one untimed warm-up launch
            if (n == 1) HIPCHK(hipEventRecord(e0, s));
            a.ucur = cur;
            a.unew = prev;
            set_acc(a, terms, 1);
            int rc2 = step_group(T, P, gr, a, s);
            if (rc2) return rc2;
            std::swap(prev, cur);
        }
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms / steps;
        return FD_OK;
    };
    for (int variant = 1; variant <= fdw::variant_count(G.ndim); ++variant) {
        const fdw::Variant v = fdw::variant_shape(G.ndim, variant);
        if (G.n2 % v.vz != 0) continue;
        std::vector<int> chunks = {0, G.n0, G.n0 / 2, G.n0 / 4, G.n0 / 8, 256, 128, 64};
        std::sort(chunks.begin(), chunks.end());
        chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
        for (int group : groups) {
            if (group > v.max_shots) continue;
            for (int chunk : chunks) {
                if (chunk != 0 && (chunk < 2 * G.r || chunk > G.n0)) continue;
                Geo T = G;
                T.variant = variant;
                T.auto_variant = false;
                T.chunk = chunk;
                T.max_group = group;
                T.variant_plain = 0;
                T.timing = nullptr;
                Scratch sc(s);
                Plan P;
                if ((rc = make_plan(T, nullptr, false, s, sc, &P))) return rc;
                Group gr = P.groups[0];
                gr.size = group;
                fdw::StepArgs a = base_args(T, P, c, 0.1);
                a.acc = acc;
                double ms_acc = 0.0, ms_plain = 0.0;
                if ((rc = time_launches(T, P, gr, a, 3, &ms_acc))) return rc;
                if ((rc = time_launches(T, P, gr, a, 0, &ms_plain))) return rc;
                const int resolved = chunk == 0 ? P.chunk : chunk;
                Best& ba = best_acc[group];
                if (ms_acc < ba.ms) ba = Best{ms_acc, variant, resolved};
                Best& bp = best_plain[group];
                if (ms_plain < bp.ms) bp = Best{ms_plain, variant, resolved};
                Best& bs = best_same[group];
                if (ms_acc + ms_plain < bs.ms) bs = Best{ms_acc + ms_plain, variant, resolved};
            }
        }
    }
    Tuned bestv;
    double best_per_shot = 1e300;
    for (int group : groups) {
        if (!best_acc.count(group) || !best_plain.count(group)) continue;
        // 2D: one shape for both launch kinds.  Separately timed shapes mispredict 2D
        // sweeps (small grids whose launches share cache-resident data): real sweeps
        // with a second shape for the plain launches ran up to 30% slower than with
        // the accumulating launches' own shape.
        const Best& ba = G.ndim == 3 ? best_acc[group] : best_same[group];
        const Best& bp = G.ndim == 3 ? best_plain[group] : best_same[group];
        const double per_pair = G.ndim == 3 ? ba.ms + bp.ms : ba.ms;
        if (per_pair / group < best_per_shot) {
            best_per_shot = per_pair / group;
            bestv.variant = ba.variant;
            bestv.chunk = ba.chunk;
            bestv.group = group;
            bestv.variant_plain = bp.variant;
            bestv.chunk_plain = bp.chunk;
            bestv.ms = per_pair / 2;
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        tune_save_locked(tune_key(G, nshot), bestv);
    }
    if (opts) *best = *opts;
    else std::memset(best, 0, sizeof(*best));
    best->variant = bestv.variant;
    best->chunk = bestv.chunk;
    best->max_group = bestv.group;
    best->variant_plain = bestv.variant_plain;
    best->chunk_plain = bestv.chunk_plain;
    if (best_ms) *best_ms = bestv.ms;
    return FD_OK;
}

// ---------------------------------------------------------------------------
// batches of independent problems
// ---------------------------------------------------------------------------

int batched(const fd_problem* probs, int nprob, double* J_host, const fd_opts* opts, hipStream_t s)
{
    if (!probs || nprob < 1) return fail(FD_E_ARG, "need at least one problem");
    if (!J_host) return fail(FD_E_ARG, "J_host is null");
    if (opts && opts->variant > 2) return fail(FD_E_ARG, "batched calls need variant 0, 1 or 2");
    Scratch sc(s);
    std::vector<Geo> G(nprob);
    std::vector<Plan> P(nprob);
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
    std::vector<const void*> cp(nprob);
    for (int p = 0; p < nprob; ++p) {
        pad_rows(&G[p]);
        if ((rc = padded_field(G[p], probs[p].c, sc, s, &cp[p]))) return rc;
    }
    int nt_max = 0;
    std::vector<fd_state> st(nprob);
    std::vector<int32_t> bstart(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        if ((rc = make_plan(G[p], &probs[p].acq, true, s, sc, &P[p]))) return rc;
        const size_t fb = G[p].ncell_pad * dsize(G[p].dtype);
        HIPCHK(sc.get(&st[p].u_a, fb));
        HIPCHK(sc.get(&st[p].u_b, fb));
        HIPCHK(sc.get(&st[p].acc, G[p].ncell_pad * dsize(G[p].acc_dtype)));
        HIPCHK(sc.get(&st[p].residual, (size_t)probs[p].nt * probs[p].acq.nrec * dsize(G[p].dtype)));
        HIPCHK(hipMemsetAsync(st[p].u_a, 0, fb, s));
        HIPCHK(hipMemsetAsync(st[p].u_b, 0, fb, s));
        HIPCHK(hipMemsetAsync(st[p].acc, 0, G[p].ncell_pad * dsize(G[p].acc_dtype), s));
        bstart[p + 1] = bstart[p] + P[p].nblk;
        nt_max = std::max(nt_max, probs[p].nt);
    }
    const int total = bstart[nprob];
    // step argument tables: forward steps n = 0..nt_max-1, backward steps aligned at
    // their ends (backward step i runs j = nt_p - 1 - i of problem p while j >= 1)
    const int nfw = nt_max, nbw = nt_max - 1;
    std::vector<fdw::StepArgs> tab((size_t)(nfw + std::max(nbw, 0)) * nprob);
    for (int p = 0; p < nprob; ++p) {
        const fd_problem& q = probs[p];
        void *prev = st[p].u_a, *cur = st[p].u_b;
        for (int n = 0; n < nfw; ++n) {
            fdw::StepArgs a = base_args(G[p], P[p], cp[p], q.dt);
            a.blk_off = P[p].groups[0].d_off;
            a.grp = P[p].groups[0].d_grp;
            a.ev = P[p].groups[0].d_ev;
            a.active = n < q.nt;
            a.acc = st[p].acc;
            set_acc(a, acc_terms(n, q.nt - 1), 1);
            a.wavelet = q.acq.wavelet;
            a.nsrc = q.acq.nsrc;
            a.sample = 1;
            a.traces = q.traces;
            a.resid = st[p].residual;
            a.obs = q.observed;
            a.nrec = q.acq.nrec;
            a.row_src = a.row_rec = std::min(n, q.nt - 1);
            a.ucur = cur;
            a.unew = prev;
            tab[(size_t)n * nprob + p] = a;
            if (n < q.nt) std::swap(prev, cur);
        }
        void *up = nullptr, *ul = nullptr;
        final_levels(st[p].u_a, st[p].u_b, q.nt, &up, &ul);
        void *vj = up, *vn = ul;
        for (int i = 0; i < nbw; ++i) {
            const int j = q.nt - 1 - i;
            fdw::StepArgs a = base_args(G[p], P[p], cp[p], q.dt);
            a.blk_off = P[p].groups[0].d_off;
            a.grp = P[p].groups[0].d_grp;
            a.ev = P[p].groups[0].d_ev;
            a.active = j >= 1;
            a.acc = st[p].acc;
            set_acc(a, acc_terms(i, q.nt - 1), -1);
            a.wavelet = q.acq.wavelet;
            a.nsrc = q.acq.nsrc;
            a.inject_rec = 1;
            a.resid = st[p].residual;
            a.nrec = q.acq.nrec;
            a.rec_scale = -q.k / q.dt;
            a.row_src = std::max(j, 1);
            a.row_rec = std::max(j - 1, 0);
            a.ucur = vj;
            a.unew = vn;
            tab[(size_t)(nfw + i) * nprob + p] = a;
            if (j >= 1) std::swap(vj, vn);
        }
    }
    fdw::StepArgs* d_tab = nullptr;
    int32_t* d_bstart = nullptr;
    HIPCHK(sc.get((void**)&d_tab, sizeof(fdw::StepArgs) * tab.size()));
    HIPCHK(sc.get((void**)&d_bstart, sizeof(int32_t) * bstart.size()));
    HIPCHK(hipMemcpyAsync(d_tab, tab.data(), sizeof(fdw::StepArgs) * tab.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_bstart, bstart.data(), sizeof(int32_t) * bstart.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));   // the host tables die with this frame

    const Geo& G0 = G[0];
    // Graph capture needs a capturable stream: the legacy null stream is not one, so
    // a graph-mode call on it works on a stream of its own (default priority), which
    // is ordered after the null stream's earlier work by the synchronisation above.
    struct OwnStream {
        hipStream_t s = nullptr;
        ~OwnStream() { if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } }
    } own;
    hipStream_t ws = s;
    if (G0.graph && s == nullptr) {
        HIPCHK(hipStreamCreate(&own.s));
        ws = own.s;
    }
    // persistent launches: barrier words (arrivals, generation, error flag), zeroed
    // here, outside any capture, and the bounded wait in device wall-clock ticks
    unsigned* d_bar = nullptr;
    long long timeout_ticks = 0;
    if (G0.persistent) {
        HIPCHK(sc.get((void**)&d_bar, 4 * sizeof(unsigned)));
        HIPCHK(hipMemsetAsync(d_bar, 0, 4 * sizeof(unsigned), s));
        HIPCHK(hipStreamSynchronize(s));
        int dev = 0, khz = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const long long us = G0.barrier_timeout_us > 0 ? G0.barrier_timeout_us : 2000000;
        timeout_ticks = std::max(1LL, us * (long long)khz / 1000);
    }
    auto barrier_ok = [&]() -> int {
        unsigned h[4] = {0, 0, 0, 0};
        HIPCHK(hipMemcpyAsync(h, d_bar, sizeof(h), hipMemcpyDeviceToHost, ws));
        HIPCHK(hipStreamSynchronize(ws));
        if (h[2] != 0)
            return fail(FD_E_DEVICE, "persistent launch: a grid barrier wait timed out (not all blocks "
                                     "could be resident); the results are invalid");
        return FD_OK;
    };
    auto sweep = [&](int first, int count) -> int {
        if (G0.persistent) {
            int grid = 0;
            HIPCHK(fdw::launch_step_persistent(G0.ndim, G0.r, G0.dtype, G0.acc_dtype, G0.variant,
                                               d_tab + (size_t)first * nprob, d_bstart, nprob, total,
                                               count, d_bar, timeout_ticks, ws, &grid));
            return FD_OK;
        }
        for (int i = 0; i < count; ++i)
            HIPCHK(fdw::launch_step_multi(G0.ndim, G0.r, G0.dtype, G0.acc_dtype, G0.variant,
                                          d_tab + (size_t)(first + i) * nprob, d_bstart, nprob, total, ws));
        return FD_OK;
    };
    // run a sweep directly, or capture it once into a graph and launch that
    auto run = [&](int first, int count, double* ms) -> int {
        SweepTimer tm(G0.timing != nullptr, ws);
        if (!G0.graph) {
            tm.start();
            if ((rc = sweep(first, count))) return rc;
            tm.stop();
        } else {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            HIPCHK(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
            int rc2 = sweep(first, count);
            hipError_t e = hipStreamEndCapture(ws, &graph);
            if ((rc2 || e != hipSuccess) && G0.persistent) {
                // this runtime cannot capture a cooperative launch: the persistent sweep is
                // a single launch anyway, so run it directly
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                g_err.clear();
                tm.start();
                if ((rc = sweep(first, count))) return rc;
                tm.stop();
                if ((rc = barrier_ok())) return rc;
                if (ms) *ms = tm.ms();
                return FD_OK;
            }
            if (rc2) { if (graph) (void)hipGraphDestroy(graph); return rc2; }
            HIPCHK(e);
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) { (void)hipGraphDestroy(graph); HIPCHK(e); }
            tm.start();
            e = hipGraphLaunch(exec, ws);
            tm.stop();
            hipError_t e2 = hipStreamSynchronize(ws);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            HIPCHK(e);
            HIPCHK(e2);
        }
        if (G0.persistent && (rc = barrier_ok())) return rc;
        if (ms) *ms = tm.ms();
        return FD_OK;
    };
    double fms = 0.0, bms = 0.0;
    if ((rc = run(0, nfw, &fms))) return rc;
    for (int p = 0; p < nprob; ++p) {
        const fd_problem& q = probs[p];
        if (q.acq.nrec == 0) continue;
        void *up = nullptr, *ul = nullptr;
        final_levels(st[p].u_a, st[p].u_b, q.nt, &up, &ul);
        HIPCHK(fdw::launch_terminal(G[p].dtype, G[p].acc_dtype, P[p].nuniq, P[p].d_ucell, P[p].d_uoff,
                                    P[p].d_uidx, P[p].d_ushot, 0, 1, G[p].ncell_pad, cp[p], 0, q.dt * q.dt,
                                    ul, up, st[p].acc,
                                    (const char*)st[p].residual +
                                        (size_t)(q.nt - 1) * q.acq.nrec * dsize(G[p].dtype),
                                    -q.k / q.dt, ws));
    }
    if (nbw > 0 && (rc = run(nfw, nbw, &bms))) return rc;
    if (ws != s) HIPCHK(hipStreamSynchronize(ws));
    if (G0.timing) {
        G0.timing->fwd_ms = fms;
        G0.timing->fwd_launches = nfw;
        G0.timing->bwd_ms = bms;
        G0.timing->bwd_launches = std::max(nbw, 0);
    }
    for (int p = 0; p < nprob; ++p) {
        const fd_problem& q = probs[p];
        if (G[p].pitch == G[p].n2) {
            HIPCHK(fdw::launch_finalize(G[p].dtype, G[p].acc_dtype, G[p].ncell, st[p].acc, q.c, 1.0 / q.k,
                                        q.grad_c, s));
        } else {   // finalise in the padded layout, then copy the rows out
            const size_t es = dsize(G[p].dtype);
            void* t = nullptr;
            HIPCHK(sc.get(&t, G[p].ncell_pad * es));
            HIPCHK(fdw::launch_finalize(G[p].dtype, G[p].acc_dtype, G[p].ncell_pad, st[p].acc, cp[p], 1.0 / q.k,
                                        t, s));
            if ((rc = copy_rows(q.grad_c, G[p].n2, t, G[p].pitch, es, (int64_t)G[p].n0 * G[p].n1, G[p].n2, s)))
                return rc;
        }
        double ss = 0.0;
        if ((rc = misfit_sum(G[p].dtype, st[p].residual, nullptr, nullptr, (int64_t)q.nt * q.acq.nrec, s,
                             sc, &ss)))
            return rc;
        J_host[p] = 0.5 * q.dt * ss;
        if (!std::isfinite(J_host[p]))
            return fail(FD_E_NONFINITE, "problem " + std::to_string(p) + ": misfit is not finite");
    }
    return FD_OK;
}

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
    const size_t es = dsize(G.dtype);
    const size_t ns = nshots > 1 ? (size_t)nshots : 1;
    const size_t nsrc = acq && acq->nsrc > 0 ? (size_t)acq->nsrc : 0;
    const size_t nrec = acq && acq->nrec > 0 ? (size_t)acq->nrec : 0;
    pad_rows(&G);   // the call's own arrays use the padded row layout
    const size_t np = (size_t)G.ncell_pad;
    size_t bytes = 2 * ns * np * es + np * 8 + (size_t)nt * nrec * es;
    if (G.pitch != G.n2) bytes += 2 * np * es;   // padded copy of c, finalisation rows
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
    bytes += 2 * plan + sizeof(double) * (3 * fdw::kReduceBlocks + 16);
    return bytes;
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
    hipStream_t s = (hipStream_t)stream;
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if ((rc = check_time(dt, nt))) return rc;
    if (!acq) return fail(FD_E_ARG, "acq is null");
    if (acq->nrec < 0) return fail(FD_E_ARG, "receiver count is negative");
    if (acq->nshot < 0) return fail(FD_E_ARG, "nshot is negative");
    if (!(k != 0.0) || !std::isfinite(k)) return fail(FD_E_ARG, "k must be finite and non-zero");
    Scratch sc(s);
    pad_rows(&G);   // the halves' own state is in the (possibly padded) row layout
    fd_state st;
    HIPCHK(sc.get(&st.u_a, G.ncell_pad * dsize(G.dtype) * nshots(acq)));
    HIPCHK(sc.get(&st.u_b, G.ncell_pad * dsize(G.dtype) * nshots(acq)));
    HIPCHK(sc.get(&st.acc, G.ncell_pad * dsize(G.acc_dtype)));
    HIPCHK(sc.get(&st.residual, (size_t)nt * acq->nrec * dsize(G.dtype)));
    if ((rc = sens_forward(grid, c, acq, dt, nt, observed, &st, traces_or_null, J_host, opts, s, true)))
        return rc;
    return sens_backward(grid, c, acq, dt, nt, k, &st, 1.0, grad_c, opts, s, true);
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

int fd_autotune(const fd_grid* grid, int32_t nshot, const fd_opts* opts, int32_t steps,
                fd_opts* best, double* best_ms, void* stream)
{
    g_err.clear();
    return autotune(grid, nshot, opts, steps, best, best_ms, (hipStream_t)stream);
}

int fd_adjoint_sensitivity_batched(const fd_problem* probs, int32_t nprob, double* J_host,
                                   const fd_opts* opts, void* stream)
{
    g_err.clear();
    return batched(probs, nprob, J_host, opts, (hipStream_t)stream);
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
