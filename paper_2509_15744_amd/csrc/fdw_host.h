// Host runtime of fdwave shared by the entry points: error state, argument checks,
// grid geometry, device scratch, launch plans (block decomposition and per-block
// event lists), the step launches and the two sweeps of Alg. 1.  The entry points
// live in fdw_api.cpp (single problems), fdw_tune.cpp (autotuner),
// fdw_batch_api.cpp (batches of problems and their plans) and fdw_design_api.cpp
// (design chain); the kernels in the .hip files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fdwave.h"
#include "fdw_internal.h"
#include "fdw_pair.h"

namespace fdh {

// Message of the last failed call in this thread (fd_last_error).
extern thread_local std::string g_err;

// Sets the message and returns `code`.
int fail(int code, const std::string& msg);

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::fdh::fail(e_ == hipErrorOutOfMemory ? FD_E_NOMEM : FD_E_DEVICE,        \
                               std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Textbook central second-derivative weights a_1..a_r of order 2, 4 or 8 (null otherwise).
const double* weights(int order);
size_t dsize(int dtype);
// The pointer must lie in a device allocation that covers `bytes` from it.
int check_dev(const void* p, size_t bytes, const char* what);

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
    bool no_partials = false;   // the caller asked for no f32 partial sums of the kernel terms
    int pairs = 0;              // two steps per launch: 1 where they fit, 0 library choice, -1 never
    int n0, n1, n2;      // internal extents (2D: n1 = 1)
    int64_t ncell;
    int pitch = 0;       // row stride of the library's own arrays (>= n2; see vd_setup)
    int64_t ncell_pad = 0;   // n0 * n1 * pitch: elements of one such array
    double dx, inv_vol;
};

// Device scratch taken stream-ordered and released at scope exit (unless handed over
// with release(), e.g. to a batch plan that keeps its tables across calls).  Given an
// arena (a fixed device array), it hands out 256-byte aligned pieces of it instead and
// never allocates; a request beyond the arena fails with hipErrorOutOfMemory.
struct Scratch {
    hipStream_t s;
    std::vector<void*> ptrs;
    char* arena = nullptr;
    size_t cap = 0, used = 0;
    explicit Scratch(hipStream_t st) : s(st) {}
    Scratch(hipStream_t st, void* base, size_t capacity) : s(st), arena((char*)base), cap(capacity) {}
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFreeAsync(p, s);
    }
    std::vector<void*> release()
    {
        std::vector<void*> out;
        out.swap(ptrs);
        return out;
    }
    hipError_t get(void** p, size_t bytes)
    {
        *p = nullptr;
        if (bytes == 0) bytes = 8;
        if (arena) {
            const size_t off = (used + 255) & ~(size_t)255;
            if (off > cap || bytes > cap - off) return hipErrorOutOfMemory;
            *p = arena + off;
            used = off + bytes;
            return hipSuccess;
        }
        hipError_t e = hipMallocAsync(p, bytes, s);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

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

// Block decomposition and events of the two-step launches (fdw_pair.hip): the tiles of
// step variant 1 (64 x 8, one cell per lane) in chunks along axis 0.  `tile` carries the
// tile events (its shot group 0); d_off_a / d_grp_a / d_ev_a list, per block and plane,
// the events in the block's ring of level n+1 (the tile and R cells around it in the
// in-plane directions, planes x0 - R .. x1 + R - 1, positions past a wall standing for
// the mirrored cell).
struct PairPlan {
    Plan tile;
    int32_t* d_off_a = nullptr;
    fdw::EvPlane* d_grp_a = nullptr;
    fdw::Event* d_ev_a = nullptr;
};

// What a sweep needs for two-step launches: the plan and a second pair of wavefields
// (ncell_pad elements each, the launches alternate between the two pairs).
struct PairSweep {
    const PairPlan* pp = nullptr;
    void* xa = nullptr;
    void* xb = nullptr;
};

// The variable-material fields of a sweep: stiffness b and its accumulator (null for
// the constant-density scheme, whose c argument is then the speed, not the mass).
struct VdFields {
    const void* stiff = nullptr;
    void* acc_b = nullptr;
    void* part_b = nullptr;   // f32 partial sums of the stiffness terms, or null
};

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

int check_grid(const fd_grid* g, const fd_opts* o, Geo* out);
int check_cells(int count, const int64_t* cells, int64_t ncell, const char* what);
int nshots(const fd_acq* a);
int check_tags(int count, const int32_t* tags, int nshot, const char* what);
int check_acq(const fd_acq* a, const Geo& G, int nt);
int src_shot(const fd_acq* a, int i);
int rec_shot(const fd_acq* a, int i);
int check_time(double dt, int nt);

// Largest stable Courant number of the leapfrog with the order-`order` stencil.
double cfl_limit(int ndim, int order);
// Speed statistics of several fields with one synchronisation, then the positivity,
// finiteness and CFL checks.
int check_speeds(const std::vector<const Geo*>& geos, const std::vector<const void*>& cs,
                 const std::vector<double>& dts, hipStream_t s, Scratch& sc);

// The remembered launch shape of (G, nshot), if any (fdw_tune.cpp).
bool apply_tuned(Geo& G, int nshot);
// Block decomposition and event tables of one problem; `pairs`: one group per shot
// carrying the shot's wavefield and its adjoint field.
int make_plan(Geo& G, const fd_acq* acq, bool want_uniq, hipStream_t s, Scratch& sc, Plan* P,
              bool pairs = false);
fdw::StepArgs base_args(const Geo& G, const Plan& P, const void* c, double dt);
int step_group(const Geo& G, const Plan& P, const Group& gr, fdw::StepArgs a, hipStream_t s);
int step(const Geo& G, const Plan& P, int gi, const fdw::StepArgs& a, hipStream_t s);
// Kernel terms of launch l of a run of `count` accumulating steps: 0, 1 (its own
// interval) or 3 (its own and the one before).
int acc_terms(int l, int count);
void set_acc(fdw::StepArgs& a, int terms, int sign);
// Whether the sweeps keep f32 partial sums of the kernel terms (f32 fields, f64
// accumulator), and a buffer for them (ncell_pad floats, or null when not).
bool use_partials(const Geo& G);
int partial_buffer(const Geo& G, Scratch& sc, void** part);
// Partial-sum mode (fdw::PM_*) of the i-th of `total` accumulating launches of a sweep.
int cycle_mode(int i, int total);
// Partial-sum mode of launch l of a run of `count` accumulating steps (the accumulating
// launches are those acc_terms marks).
int part_mode(int l, int count);
// acc_terms and, when a.part is set, part_mode of launch l, with the sign of the sweep.
void set_acc_at(fdw::StepArgs& a, int l, int count, int sign);
// Partial-sum mode of the stiffness terms of launch l of a sweep of nlaunch launches
// (variable material: every launch adds them).
void set_face_at(fdw::StepArgs& a, int l, int nlaunch);

int prepare(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int nt,
            const fd_opts* opts, hipStream_t s, Scratch& sc, Geo* G, bool stats);
// `part`: a partial-sum buffer of ncell_pad floats for the kernel terms (f32 fields with
// an f64 accumulator, constant density only), or null to add them to acc directly.
// `pw`: run the steps two per launch where pw->pp is set (constant density).
int forward_sweep(const Geo& G, const Plan& P, const void* c, const fd_acq* acq, double dt, int nt,
                  const void* obs, void* ua, void* ub, void* acc, void* resid, void* traces,
                  hipStream_t s, const VdFields& vd = VdFields(), void* part = nullptr,
                  const PairSweep* pw = nullptr);
void final_levels(void* ua, void* ub, int nt, void** prev, void** cur);
int backward_sweep(const Geo& G, const Plan& P, const void* c, const fd_acq* acq, double dt, int nt,
                   double k, void* ua, void* ub, void* acc, void* resid, hipStream_t s,
                   const VdFields& vd = VdFields(), void* part = nullptr, const PairSweep* pw = nullptr);
// Whether the sweeps of (G, acq) run two steps per launch: 3D, one shot, every extent
// at least twice the stencil radius, asked for (G.pairs > 0).
bool use_pairs(const Geo& G, const fd_acq* acq);
// The plan of the two-step launches (G with rows already padded) and, with ws, the
// second pair of wavefields.
int make_pair_sweep(const Geo& G, const fd_acq* acq, hipStream_t s, Scratch& sc, PairPlan* PP, PairSweep* ws);
// Fixed-order sum of (x - y)^2 (x^2 when y is null) into *out (host); synchronises.
int misfit_sum(int dtype, const void* x, const void* y, void* diff, int64_t n, hipStream_t s,
               Scratch& sc, double* out);

void pad_rows(Geo* G);
int copy_rows(void* dst, int64_t dpitch, const void* src, int64_t spitch, size_t es, int64_t rows, int64_t n2,
              hipStream_t s);
int padded_field(const Geo& G, const void* f, Scratch& sc, hipStream_t s, const void** fp);
int padded_material(const Geo& G, const void* m, const void* b, Scratch& sc, hipStream_t s, const void** mp,
                    const void** bp);
int vd_work(const Geo& G, const fd_state* st, void* acc_b, int ns, bool own_state, bool copy_in, Scratch& sc,
            hipStream_t s, VdWork* w);
int work_out(const Geo& G, const VdWork& w, const fd_state* st, void* acc_b, int ns, hipStream_t s);
int check_state(const fd_state* st, const Geo& G, int nt, const fd_acq* acq);

}  // namespace fdh
