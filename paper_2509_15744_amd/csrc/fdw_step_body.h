// The fused leapfrog step of fdwave for gfx950 (CDNA4, wave64): the per-tile body
// shared by the single-problem, multi-problem and persistent kernels.
//
// One step of the scheme (paper Sec. 3.1, Eq. FDstencil2 with rho^-1 = 1,
// kappa = c^2, order-2r Laplacian) over the whole grid, fused with the work that
// Alg. 1 does per time step: source injection, receiver sampling, the residual /
// adjoint force and the kernel increments, K(u,u) in the forward loop and K(v,v)
// in the superposed backward loop (or, for the exact re-simulation sweep, the
// cross term of u and the adjoint field).  One launch per time step; 2D and 3D
// share the code.
//
// Layout of the work:
//  * a block owns a tile of the planes normal to axis 0 (3D: TY x WZ cells of
//    axes 1 and 2; 2D: WZ cells of axis 1) and marches along axis 0 through a
//    chunk of planes;
//  * a lane owns VZ consecutive cells of the contiguous axis (WZ = 64 VZ per
//    wave row), so every global access of a wave is one coalesced row segment
//    of 256 VZ bytes (f32) issued as dword, dwordx2 or dwordx4 loads;
//  * a lane advances S shots of the same medium at once: c and the shared
//    accumulator are read once per cell for all S wavefields;
//  * each lane keeps the 2r+1 values of its column along axis 0 in registers
//    (a rotating queue), so axis-0 neighbours cost no extra reads;
//  * the current plane is staged in LDS with an r-wide halo for the in-plane
//    neighbours (cross-shaped stencil: no corner halo), double-buffered so one
//    barrier per plane suffices;
//  * software pipelining: every load of plane x+1 (queue entry x+1+r, halo,
//    u^{n-1}, c, accumulator) is issued before plane x is computed, so a whole
//    plane of work covers the memory latency;
//  * plane bases are wave-uniform 64-bit pointers, in-plane offsets 32-bit;
//  * u^{n+1} overwrites u^{n-1} in place and the speed c is read instead of a
//    stored dt^2 c^2 array, so a step streams four arrays; those streams are read
//    and written non-temporally, which leaves the cache to the u^n halos;
//  * block ids are remapped so that consecutive tiles run on the same XCD
//    (dispatch is round-robin over the 8 XCDs) and share halo rows in its L2;
//  * with f32 fields and an f64 accumulator, most accumulating launches add their
//    kernel terms to an f32 partial sum per cell instead of the accumulator, which
//    takes it in every kPartialCycle-th of them (part_mode).
//
// Difference form of the Laplacian, sum_j w_j [(u_{+j} - u_0) + (u_{-j} - u_0)]:
// L applied to a constant is exactly zero in f32 even though the rounded weights
// do not sum to zero, which removes the phase drift of the a_0 form.

#pragma once

#include <hip/hip_runtime.h>

#include "fdw_internal.h"

// qualifier of pointers into device (global) memory
#define GLOBAL_AS __attribute__((address_space(1)))

namespace fdw {


// Ghost index: half-sample mirror about the wall faces, then clamped into the
// array (the clamp only matters for tile-overhang lanes, which store nothing).
__device__ __forceinline__ int ghost(int i, int n)
{
    i = i < 0 ? -1 - i : i;
    i = i >= n ? 2 * n - 1 - i : i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <typename T, int V>
struct Vec { typedef T __attribute__((ext_vector_type(V))) type; };
template <typename T>
struct Vec<T, 1> { typedef T type; };

template <typename T, int V>
__device__ __forceinline__ T el(const typename Vec<T, V>::type& v, int i)
{
    if constexpr (V == 1) return v;
    else return v[i];
}
template <typename T, int V>
__device__ __forceinline__ void set_el(typename Vec<T, V>::type& v, int i, T x)
{
    if constexpr (V == 1) v = x;
    else v[i] = x;
}

template <typename T, int V>
__device__ __forceinline__ typename Vec<T, V>::type reversed(const typename Vec<T, V>::type& v)
{
    if constexpr (V == 1) return v;
    else if constexpr (V == 2) return __builtin_shufflevector(v, v, 1, 0);
    else return __builtin_shufflevector(v, v, 3, 2, 1, 0);
}

// V consecutive cells of one row starting at z (z and the row length n2 are multiples
// of V), without a branch around the load.  A lane past the wall (z >= n2) reads the
// aligned vector that holds its mirrored ghost cells and, when MIRROR, reverses it:
// cell z + i maps to 2 n2 - 1 - z - i.  Without MIRROR such lanes get in-bounds values
// they never use.
template <typename T, int V, bool STREAM, bool MIRROR, typename PTR>
__device__ __forceinline__ typename Vec<T, V>::type load_row(PTR row, int z, int n2)
{
    typedef typename Vec<T, V>::type vec;
    const bool past = z >= n2;
    const int zs = max(past ? 2 * n2 - z - V : z, 0);
    vec v;
    if constexpr (STREAM) v = __builtin_nontemporal_load((const vec*)(row + zs));
    else v = *(const vec*)(row + zs);
    if constexpr (MIRROR && V > 1) v = past ? reversed<T, V>(v) : v;
    return v;
}

// Compile-time shape of one kernel variant.
template <int R, typename T, int NDIM, int TZ, int TY, int RY, int VZ, int S>
struct Shape {
    static constexpr int TYT = TY / RY;            // thread rows; a thread owns RY tile rows
    static constexpr int NT = TZ * TYT;            // threads per block
    static constexpr int WZ = TZ * VZ;             // tile width in cells
    static constexpr int RYH = (NDIM == 3) ? R : 0;
    static constexpr int PADL = VZ * ((R + VZ - 1) / VZ);   // left pad keeps rows VZ-aligned
    static constexpr int LZ = PADL + WZ + PADL;
    static constexpr int LSZ = (TY + 2 * RYH) * LZ;          // one plane of one shot
    static constexpr int HYV = (NDIM == 3) ? 2 * R * TZ : 0; // halo row vectors above and below
    static constexpr int HZ = 2 * R * TY;                    // halo cells left and right
    static constexpr int NHY = (HYV + NT - 1) / NT;
    static constexpr int NHZ = (HZ + NT - 1) / NT;
    static constexpr int NHY1 = NHY > 0 ? NHY : 1;
    static constexpr int LDS = 2 * S * LSZ;                  // double buffer, all shots
};

// ---------------------------------------------------------------------------
// sources and receivers of a block, plane by plane
// ---------------------------------------------------------------------------

// One plane's events staged in LDS, double-buffered by plane parity like the planes.
template <typename T>
struct EventStage {
    int32_t key[2][kStagedEvents];   // lane << 8 | kind (kind = shot slot << 1 | source/receiver)
    int32_t idx[2][kStagedEvents];   // source or receiver number
    T val[2][kStagedEvents];         // injected value: wavelet / dx^d, or rec_scale * residual
    T obs[2][kStagedEvents];         // observed value at a receiver (forward sampling)
};

// A block's walk over its plane groups (all fields block-uniform).  The next group
// is read one plane group ahead; plane x's events are ev[ea, e).  Planes may be
// negative (the two-step launches walk mirrored planes past the wall at x = 0), so an
// exhausted walk holds kNoPlane, which no plane equals, and an empty range.
constexpr int kNoPlane = -2147483647 - 1;

__device__ __forceinline__ EvPlane no_plane()
{
    EvPlane g;
    g.plane = kNoPlane;
    g.begin = g.end = g.pad = 0;
    return g;
}

// Group i and event i of the tables in device memory (global loads, field by field).
__device__ __forceinline__ EvPlane read_group(const EvPlane* grp, int i)
{
    const GLOBAL_AS int32_t* q = (const GLOBAL_AS int32_t*)(grp + i);
    EvPlane g;
    g.plane = q[0];
    g.begin = q[1];
    g.end = q[2];
    g.pad = q[3];
    return g;
}
__device__ __forceinline__ Event read_event(const Event* ev, int i)
{
    const GLOBAL_AS int32_t* q = (const GLOBAL_AS int32_t*)(ev + i);
    Event e;
    e.plane = q[0];
    e.lane = q[1];
    e.kind = q[2];
    e.idx = q[3];
    return e;
}

struct PlaneEvents {
    int gi, g_end;
    EvPlane next;
    int ea, e, eb;
    bool has, staged;
};

__device__ __forceinline__ void events_begin(PlaneEvents& pe, const StepArgs& a, int b)
{
    pe.gi = ((const GLOBAL_AS int32_t*)a.blk_off)[b];
    pe.g_end = ((const GLOBAL_AS int32_t*)a.blk_off)[b + 1];
    pe.next = pe.gi < pe.g_end ? read_group(a.grp, pe.gi) : no_plane();
}

// Finds plane x's events and, when they fit, stages them with their values (all
// threads of the block take part; the caller's barrier publishes them).
template <typename T, int NT>
__device__ __forceinline__ void events_at_plane(PlaneEvents& pe, const StepArgs& a, EventStage<T>& st,
                                                int x, int tid)
{
    pe.has = pe.next.plane == x;
    pe.ea = 0;
    pe.e = 0;
    pe.staged = false;
    pe.eb = x & 1;
    if (!pe.has) return;
    pe.ea = pe.next.begin;
    pe.e = pe.next.end;
    pe.next = ++pe.gi < pe.g_end ? read_group(a.grp, pe.gi) : no_plane();
    pe.staged = pe.e - pe.ea <= kStagedEvents;
    if (!pe.staged) return;
    for (int t = tid; t < pe.e - pe.ea; t += NT) {
        const Event ev = read_event(a.ev, pe.ea + t);
        T v = (T)0, o = (T)0;
        if (ev_kind(ev.kind) == EV_SRC) {
            v = ((const GLOBAL_AS T*)a.wavelet)[(int64_t)a.row_src * a.nsrc + ev.idx] * (T)a.inv_vol;
        } else {
            const int64_t r = (int64_t)a.row_rec * a.nrec + ev.idx;
            if (a.inject_rec) v = (T)a.rec_scale * ((const GLOBAL_AS T*)a.resid)[r];
            if (a.sample && a.resid) o = ((const GLOBAL_AS T*)a.obs)[r];
        }
        st.key[pe.eb][t] = (ev.lane << 8) | ev.kind;
        st.idx[pe.eb][t] = ev.idx;
        st.val[pe.eb][t] = v;
        st.obs[pe.eb][t] = o;
    }
}

// First staged event of plane slot eb whose key is at least k: the keys ascend within
// a plane (the events are sorted by lane, then kind), so a lane can find its own events
// by bisection instead of scanning every event of the plane.  Measured, this pays in 2D
// (rows that hold many shots' sources or a receiver line: +6% on 32 shots of 2048²)
// and costs in 3D (planes with few events, where the longer code slowed the 1024³
// sweep by 1.7%), so the 3D kernels keep the scan (BISECT = false below).
template <typename T>
__device__ __forceinline__ int first_key(const EventStage<T>& st, int eb, int n, int k)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st.key[eb][mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Point force at tile lane `lane`, shot slot s of this plane: the sources there and,
// when injecting, the receivers, summed in event order.
template <bool BISECT, typename T>
__device__ __forceinline__ T point_force(const PlaneEvents& pe, const StepArgs& a,
                                         const EventStage<T>& st, int lane, int s)
{
    T f = (T)0;
    if (pe.staged) {
        const int n = pe.e - pe.ea;
        const int want = ((lane << 8) | (s << 1)) >> 1;
        for (int t = BISECT ? first_key(st, pe.eb, n, lane << 8) : 0; t < n; ++t) {
            const int key = st.key[pe.eb][t];
            if (BISECT && (key >> 8) != lane) break;
            if ((key >> 1) == want && ((key & 1) == EV_SRC || a.inject_rec)) f += st.val[pe.eb][t];
        }
    } else {
        for (int v = pe.ea; v < pe.e; ++v) {
            const Event ev = read_event(a.ev, v);
            if (ev.lane != lane || ev_shot(ev.kind) != s) continue;
            if (ev_kind(ev.kind) == EV_SRC)
                f += ((const GLOBAL_AS T*)a.wavelet)[(int64_t)a.row_src * a.nsrc + ev.idx] * (T)a.inv_vol;
            else if (a.inject_rec)
                f += (T)a.rec_scale * ((const GLOBAL_AS T*)a.resid)[(int64_t)a.row_rec * a.nrec + ev.idx];
        }
    }
    return f;
}

// Trace and residual of the receivers at lane `lane`, shot slot s, for the new level.
template <bool BISECT, typename T>
__device__ __forceinline__ void sample_receivers(const PlaneEvents& pe, const StepArgs& a,
                                                 const EventStage<T>& st, int lane, int s, T uni)
{
    if (pe.staged) {
        const int n = pe.e - pe.ea;
        const int want = (lane << 8) | (s << 1) | EV_REC;
        for (int t = BISECT ? first_key(st, pe.eb, n, want) : 0; t < n; ++t) {
            if (st.key[pe.eb][t] != want) {
                if (BISECT) break;
                continue;
            }
            const int64_t o = (int64_t)a.row_rec * a.nrec + st.idx[pe.eb][t];
            if (a.traces) ((GLOBAL_AS T*)a.traces)[o] = uni;
            if (a.resid) ((GLOBAL_AS T*)a.resid)[o] = uni - st.obs[pe.eb][t];
        }
    } else {
        for (int v = pe.ea; v < pe.e; ++v) {
            const Event ev = read_event(a.ev, v);
            if (ev.lane != lane || ev.kind != (EV_REC | (s << 1))) continue;
            const int64_t o = (int64_t)a.row_rec * a.nrec + ev.idx;
            if (a.traces) ((GLOBAL_AS T*)a.traces)[o] = uni;
            if (a.resid) ((GLOBAL_AS T*)a.resid)[o] = uni - ((const GLOBAL_AS T*)a.obs)[o];
        }
    }
}

// One block's share of one step: logical block b of problem `a`.  ACC = false compiles
// a launch that never touches the accumulator (no registers held for it, which lets
// more waves stay resident); with ACC = true a.acc_sign decides at run time.
template <int R, typename T, typename AT, int NDIM, int TZ, int TY, int RY, int VZ, int S,
          bool ACC = true>
__device__ __forceinline__ void step_body(const StepArgs& a, const int b, T* __restrict__ lds)
{
    typedef Shape<R, T, NDIM, TZ, TY, RY, VZ, S> SH;
    typedef typename Vec<T, VZ>::type vec;
    typedef typename Vec<AT, VZ>::type avec;
    typedef typename Vec<float, VZ>::type pvec;
    constexpr int TYT = SH::TYT, NT = SH::NT, WZ = SH::WZ, RYH = SH::RYH, PADL = SH::PADL;
    constexpr int LZ = SH::LZ, LSZ = SH::LSZ, HYV = SH::HYV, HZ = SH::HZ;
    constexpr int NHY = SH::NHY, NHZ = SH::NHZ, NHY1 = SH::NHY1;

    const int tzb = b % a.ntz;
    const int rest = b / a.ntz;
    const int tyb = rest % a.nty;
    const int chb = rest / a.nty;

    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int z0 = tzb * WZ, y0 = tyb * TY;
    const int x0 = chb * a.chunk_len;
    const int x1 = min(x0 + a.chunk_len, n0);
    const int tid = threadIdx.x;
    const int lz = tid % TZ;
    const int lyt = tid / TZ;
    const int z = z0 + lz * VZ;              // first cell of this lane
    const bool zlive = z < n2;
    const int pitch = a.pitch;                  // row stride (rows may be padded)
    const int64_t ps = (int64_t)n1 * pitch;
    const int64_t sst = a.shot_stride;

    // the buffers are device memory: pointers in the global address space give global
    // loads even when `a` was read from a table in memory (generic pointers would give
    // flat loads, whose waits also wait for the LDS traffic and serialise the
    // plane-ahead loads with the plane's LDS work)
    const GLOBAL_AS T* __restrict__ ucur = (const GLOBAL_AS T*)a.ucur;
    GLOBAL_AS T* __restrict__ unew = (GLOBAL_AS T*)a.unew;
    const GLOBAL_AS T* __restrict__ cc = (const GLOBAL_AS T*)a.c;
    GLOBAL_AS AT* __restrict__ acc = (GLOBAL_AS AT*)a.acc;
    const bool use_acc = ACC && a.acc_sign != 0;
    // f32 partial sums of the kernel terms exist for f32 fields with an f64 accumulator
    constexpr bool PARTS = ACC && sizeof(T) == 4 && sizeof(AT) == 8;
    GLOBAL_AS float* __restrict__ part = (GLOBAL_AS float*)a.part;
    const int pmode = (PARTS && use_acc) ? a.part_mode : PM_DIRECT;
    const bool rd_acc = use_acc && (pmode == PM_DIRECT || pmode == PM_FLUSH);
    const bool rd_part = PARTS && use_acc && (pmode == PM_ADD || pmode == PM_FLUSH);
    const bool wr_part = PARTS && use_acc && (pmode == PM_START || pmode == PM_ADD);
    T w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) w[j] = (T)a.w[j];
    const T dt2 = (T)a.dt2;

    // own cells: row offset within a plane (ghosted for overhang rows, which never store)
    int roff[RY], lofs[RY], lane0[RY];
    bool live[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        const int ly = lyt + k * TYT;
        const int y = y0 + ly;
        roff[k] = ghost(y, n1) * pitch;
        live[k] = zlive && (y < n1);
        lofs[k] = (ly + RYH) * LZ + PADL + lz * VZ;
        lane0[k] = ly * WZ + lz * VZ;
    }
    // halo rows (3D): LDS slot of the vector and its row offset in the plane
    int hyl[NHY1], hyr[NHY1], hyz[NHY1];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int h = tid + i * NT;
        const int row = h / TZ;
        const int sy = row < R ? row : row + TY;
        const int cz = (h % TZ) * VZ;
        hyl[i] = h < HYV ? sy * LZ + PADL + cz : -1;
        hyr[i] = ghost(y0 + sy - R, n1) * pitch;
        hyz[i] = z0 + cz;
    }
    // halo columns: LDS slot and in-plane offset of single cells
    int hzl[NHZ], hzg[NHZ];
#pragma unroll
    for (int i = 0; i < NHZ; ++i) {
        const int h = tid + i * NT;
        const int row = h / (2 * R);
        const int col = h % (2 * R);
        const int sz = col < R ? PADL - R + col : PADL + WZ + (col - R);
        hzl[i] = h < HZ ? (RYH + row) * LZ + sz : -1;
        const int gy = ghost(y0 + (h < HZ ? row : 0), n1);
        hzg[i] = gy * pitch + ghost(z0 + sz - PADL, n2);
    }

    // register queue along axis 0: q[s][k][R + d] = u^n(x + d) of shot s, d in [-R, R]
    vec q[S][RY][2 * R + 1];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int k = 0; k < RY; ++k)
#pragma unroll
            for (int d = 0; d < 2 * R + 1; ++d)
                q[s][k][d] = load_row<T, VZ, false, true>(
                    ucur + s * sst + (int64_t)ghost(x0 - R + d, n0) * ps + roff[k], z, n2);

    // operands of one plane xp: the queue entry u^n(xp + R), u^{n-1}, c, accumulator
    // and partial sums of the own cells, and the in-plane halo of u^n
    struct PlaneOps {
        vec q[S][RY], u[S][RY], v[RY], hy[S][NHY1];
        avec a[RY];
        pvec pt[RY];
        T hz[S][NHZ];
    };
    auto load_ops = [&](PlaneOps& o, int xp, bool with_q) {
        const int64_t xn = (int64_t)xp * ps;
        const int64_t xq = (int64_t)ghost(xp + R, n0) * ps;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (with_q) o.q[s][k] = load_row<T, VZ, false, true>(ucur + s * sst + xq + roff[k], z, n2);
                o.u[s][k] = load_row<T, VZ, true, false>(unew + s * sst + xn + roff[k], z, n2);
            }
            o.v[k] = load_row<T, VZ, true, false>(cc + xn + roff[k], z, n2);
            if (rd_acc) o.a[k] = load_row<AT, VZ, true, false>(acc + xn + roff[k], z, n2);
            if (rd_part) o.pt[k] = load_row<float, VZ, true, false>(part + xn + roff[k], z, n2);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int i = 0; i < NHY; ++i)
                if (hyl[i] >= 0) o.hy[s][i] = load_row<T, VZ, false, true>(ucur + s * sst + xn + hyr[i], hyz[i], n2);
#pragma unroll
            for (int i = 0; i < NHZ; ++i) o.hz[s][i] = hzl[i] >= 0 ? ucur[s * sst + xn + hzg[i]] : (T)0;
        }
    };

    // plane-x operands (its queue entry is already in q); those of plane x + 1 load
    // while plane x computes
    PlaneOps cur, next;
    load_ops(cur, x0, false);

    // events: a plane's sources and receivers (and their wavelet, adjoint force and
    // observed values) are staged in LDS, so lanes find theirs without global loads
    __shared__ EventStage<T> est;
    PlaneEvents pe;
    events_begin(pe, a, b);

    for (int x = x0; x < x1; ++x) {
        const int64_t xo = (int64_t)x * ps;
        const bool more = x + 1 < x1;
        if (more) load_ops(next, x + 1, true);

        // stage plane x of every shot
#pragma unroll
        for (int s = 0; s < S; ++s) {
            T* L = lds + ((x & 1) * S + s) * LSZ;
#pragma unroll
            for (int k = 0; k < RY; ++k) *(vec*)(L + lofs[k]) = q[s][k][R];
#pragma unroll
            for (int i = 0; i < NHY; ++i)
                if (hyl[i] >= 0) *(vec*)(L + hyl[i]) = cur.hy[s][i];
#pragma unroll
            for (int i = 0; i < NHZ; ++i)
                if (hzl[i] >= 0) L[hzl[i]] = cur.hz[s][i];
        }
        events_at_plane<T, NT>(pe, a, est, x, tid);
        __syncthreads();

#pragma unroll
        for (int k = 0; k < RY; ++k) {
            if (!live[k]) continue;
            const int s0 = lofs[k];
            vec un[S];
            avec an;
            pvec pn;
            const T* L0 = lds + (x & 1) * S * LSZ;
#pragma unroll
            for (int i = 0; i < VZ; ++i) {
                const T cvi = el<T, VZ>(cur.v[k], i);
                const T coef = a.coef_direct ? cvi : dt2 * cvi * cvi;
                AT dsum = (AT)0, dpair = (AT)0, dpair_p = (AT)0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const T* L = L0 + s * LSZ;
                    const T u0 = el<T, VZ>(q[s][k][R], i);
                    T lap = (T)0;
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap += w[j - 1] * ((el<T, VZ>(q[s][k][R + j], i) - u0) + (el<T, VZ>(q[s][k][R - j], i) - u0));
                    if (NDIM == 3) {
#pragma unroll
                        for (int j = 1; j <= R; ++j)
                            lap += w[j - 1] * ((L[s0 + i + j * LZ] - u0) + (L[s0 + i - j * LZ] - u0));
                    }
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap += w[j - 1] * ((L[s0 + i + j] - u0) + (L[s0 + i - j] - u0));

                    if (pe.has) lap += point_force<NDIM == 2>(pe, a, est, lane0[k] + i, s);

                    const T uni = (u0 + u0) - el<T, VZ>(cur.u[s][k], i) + coef * lap;
                    set_el<T, VZ>(un[s], i, uni);
                    // kernel terms: the interval this launch completes and, with acc_prev,
                    // the one before it (its two ends are already in registers)
                    const AT d = (AT)(uni - u0);
                    const AT dp = a.acc_prev ? (AT)(u0 - el<T, VZ>(cur.u[s][k], i)) : (AT)0;
                    if (a.acc_cross) {   // exact re-simulation: slots (2p, 2p+1) hold (u, mu)
                        if (s & 1) dsum += dpair * d + dpair_p * dp;
                        else { dpair = d; dpair_p = dp; }
                    } else {
                        // one explicit rounding order, which the two-step launches repeat
                        dsum += fma(d, d, dp * dp);
                    }
                    if (a.sample && pe.has) sample_receivers<NDIM == 2>(pe, a, est, lane0[k] + i, s, uni);
                }
                if (rd_acc) {
                    const AT tot = rd_part ? dsum + (AT)el<float, VZ>(cur.pt[k], i) : dsum;
                    const AT ai = el<AT, VZ>(cur.a[k], i);
                    set_el<AT, VZ>(an, i, a.acc_sign > 0 ? ai + tot : ai - tot);
                }
                if (wr_part) {
                    const AT tot = rd_part ? dsum + (AT)el<float, VZ>(cur.pt[k], i) : dsum;
                    set_el<float, VZ>(pn, i, (float)tot);
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s)
                __builtin_nontemporal_store(un[s], (vec*)(unew + s * sst + xo + roff[k] + z));
            if (rd_acc) __builtin_nontemporal_store(an, (avec*)(acc + xo + roff[k] + z));
            if (wr_part) __builtin_nontemporal_store(pn, (pvec*)(part + xo + roff[k] + z));
        }

        // rotate to plane x + 1
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k)
#pragma unroll
                for (int s = 0; s < S; ++s) {
#pragma unroll
                    for (int d = 0; d < 2 * R; ++d) q[s][k][d] = q[s][k][d + 1];
                    q[s][k][2 * R] = next.q[s][k];
                }
            cur = next;
        }
    }
}

// XCD-aware logical block id: hardware block i runs on XCD i % 8, so consecutive
// logical blocks (neighbouring tiles) go to the same XCD.
__device__ __forceinline__ int logical_block(int nblk)
{
    const int per = (nblk + 7) >> 3;
    const int hb = blockIdx.x;
    return (hb & 7) * per + (hb >> 3);
}

}  // namespace fdw
