// Two time steps per launch (temporal blocking along the marching axis) for the
// constant-density 3D step of fdwave: one launch reads u^{n-1}, u^n and c once and
// writes u^{n+1} and u^{n+2} to a second pair of arrays, with the kernel terms of both
// intervals it completes, so a sweep streams 28 instead of 40 bytes per cell for two
// steps (f32 fields, f32 partial sums of the kernel terms).
//
// A block owns a TY x WZ tile of the planes normal to axis 0 (one cell per lane) and
// marches along axis 0.  At plane xl it computes level n+1 on the tile and on a ring
// of width R around it in the in-plane directions (the cross-shaped region the
// order-2R stencil of level n+2 reads: R rows above and below the tile over its width,
// R columns left and right over its height); R planes behind, at x2 = xl - R, it
// computes level n+2 on the tile.  The ring values are recomputed by the neighbouring
// tiles' blocks with the same arithmetic (a position past a wall mirrors the cell it
// stands for, and the position-based stencil there adds the same pairs of neighbours
// as the cell's own, in swapped order), so both levels equal those of two one-step
// launches bit for bit.  Level n+1 runs over planes x0 - R .. x1 + R - 1 of the
// block's chunk [x0, x1) (planes past a wall are the mirrored ones); the output of
// each level is stored on the tile's own planes only.
//
// Registers: per thread the axis-0 queue of u^n (2R + 1 planes) for its tile cell, its
// ring cell above or below (threads < 2R WZ) and its ring cell left or right (threads
// < 2R TY), the queue of u^{n+1} for its tile cell (2R + 1), the last R ring values of
// u^{n+1}, and the last R + 1 planes of c of its tile cell.  LDS: the current plane of
// u^n over the tile and a 2R-wide in-plane halo (cross plus the ring's corners), the
// plane x2 of u^{n+1} over the tile and an R-wide halo (cross), both double-buffered so
// one barrier per plane suffices, and the staged events of three walks (ring events of
// level n+1, tile events of level n+1 sampled at x2, tile events of level n+2).

#include "fdw_pair.h"
#include "fdw_step_body.h"

namespace fdw {

template <int R>
struct PairShape {
    static constexpr int TZ = kPairTZ, TY = kPairTY, NT = TZ * TY, WZ = TZ;
    static constexpr int Z0 = WZ + 4 * R, Y0 = TY + 4 * R;   // u^n plane, offsets -2R
    static constexpr int Z1 = WZ + 2 * R, Y1 = TY + 2 * R;   // u^{n+1} plane, offsets -R
    static constexpr int NSTRIP = 2 * R * WZ;                 // ring cells above and below
    static constexpr int NSIDE = 2 * R * TY;                  // ring cells left and right
    static constexpr int NHALO = 2 * R * WZ + 4 * R * R + 2 * R * TY;   // u^n halo of the ring
    static constexpr int NH = (NHALO + NT - 1) / NT;
    static_assert(NSTRIP <= NT && NSIDE <= NT, "one ring cell of each kind per thread");
};

// In-plane position (sy, sz) of halo cell h of the u^n plane, relative to the tile
// origin: the 2R-deep rows beyond the ring above and below (tile width), the ring's
// corners, the 2R-deep columns beyond the ring left and right (tile height).
template <int R>
__device__ __forceinline__ void halo_pos(int h, int& sy, int& sz)
{
    typedef PairShape<R> SH;
    if (h < 2 * R * SH::WZ) {
        const int fr = h / SH::WZ;
        sz = h % SH::WZ;
        sy = fr < R ? fr - 2 * R : SH::TY + R + (fr - R);
        return;
    }
    h -= 2 * R * SH::WZ;
    if (h < 4 * R * R) {
        const int corner = h / (R * R), rem = h % (R * R);
        sy = (corner & 1) ? SH::TY + rem / R : rem / R - R;
        sz = (corner & 2) ? SH::WZ + rem % R : rem % R - R;
        return;
    }
    h -= 4 * R * R;
    const int side = h / (R * SH::TY), rem = h % (R * SH::TY);
    sy = rem / R;
    sz = side ? SH::WZ + R + rem % R : rem % R - 2 * R;
}

template <int R, typename T, typename AT, bool ACC>
__global__ __launch_bounds__(512) void pair_kernel(PairArgs p)
{
    typedef PairShape<R> SH;
    constexpr int TZ = SH::TZ, TY = SH::TY, NT = SH::NT, WZ = SH::WZ;
    constexpr int Z0 = SH::Z0, Z1 = SH::Z1;
    constexpr int NH = SH::NH;
    __shared__ __attribute__((aligned(16))) T lds0[2][SH::Y0 * Z0];
    __shared__ __attribute__((aligned(16))) T lds1[2][SH::Y1 * Z1];
    __shared__ EventStage<T> est_a, est_b1, est_b2;

    const StepArgs& a = p.s;
    const int b = logical_block(a.nblk);
    if (b >= a.nblk) return;
    const int tzb = b % a.ntz;
    const int rest = b / a.ntz;
    const int tyb = rest % a.nty;
    const int chb = rest / a.nty;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int z0 = tzb * WZ, y0 = tyb * TY;
    const int x0 = chb * a.chunk_len;
    const int x1 = min(x0 + a.chunk_len, n0);
    const int tid = threadIdx.x;
    const int pitch = a.pitch;
    const int64_t ps = (int64_t)n1 * pitch;

    const T* __restrict__ uprev = (const T*)a.unew;   // u^{n-1}
    const T* __restrict__ ucur = (const T*)a.ucur;    // u^n
    T* __restrict__ out1 = (T*)p.out1;                 // u^{n+1}
    T* __restrict__ out2 = (T*)p.out2;                 // u^{n+2}
    const T* __restrict__ cc = (const T*)a.c;
    AT* __restrict__ acc = (AT*)a.acc;
    float* __restrict__ part = (float*)a.part;
    T w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) w[j] = (T)a.w[j];
    const T dt2 = (T)a.dt2;

    // accumulation of this launch: terms 0, 1 (interval n, n+1 alone) or 3 (both)
    const int terms = ACC ? p.terms : 0;
    constexpr bool PARTS = ACC && sizeof(T) == 4 && sizeof(AT) == 8;
    const int pmode = (PARTS && terms) ? a.part_mode : PM_DIRECT;
    const bool rd_acc = terms && (pmode == PM_DIRECT || pmode == PM_FLUSH);
    const bool rd_part = PARTS && terms && (pmode == PM_ADD || pmode == PM_FLUSH);
    const bool wr_part = PARTS && terms && (pmode == PM_START || pmode == PM_ADD);

    // this thread's cells: tile (t), ring above/below (s), ring left/right (d)
    const int ty = tid / TZ, tz = tid % TZ;
    const bool has_s = tid < SH::NSTRIP, has_d = tid < SH::NSIDE;
    int sy_s = 0, sz_s = 0, sy_d = 0, sz_d = 0;
    if (has_s) {
        const int sr = tid / WZ;
        sz_s = tid % WZ;
        sy_s = sr < R ? sr - R : TY + (sr - R);
    }
    if (has_d) {
        const int side = tid / (R * TY), rem = tid % (R * TY);
        sy_d = rem / R;
        sz_d = side ? WZ + rem % R : rem % R - R;
    }
    const int off_t = ghost(y0 + ty, n1) * pitch + ghost(z0 + tz, n2);
    const int off_s = ghost(y0 + sy_s, n1) * pitch + ghost(z0 + sz_s, n2);
    const int off_d = ghost(y0 + sy_d, n1) * pitch + ghost(z0 + sz_d, n2);
    const bool live = (y0 + ty < n1) && (z0 + tz < n2);
    const int l0_t = (ty + 2 * R) * Z0 + tz + 2 * R;
    const int l0_s = (sy_s + 2 * R) * Z0 + sz_s + 2 * R;
    const int l0_d = (sy_d + 2 * R) * Z0 + sz_d + 2 * R;
    const int l1_t = (ty + R) * Z1 + tz + R;
    const int l1_s = (sy_s + R) * Z1 + sz_s + R;
    const int l1_d = (sy_d + R) * Z1 + sz_d + R;
    const int lane_t = ty * WZ + tz;                    // lanes of the ring walk
    const int lane_s = TY * WZ + tid;
    const int lane_d = TY * WZ + SH::NSTRIP + tid;
    int hl[NH], hg[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int h = tid + i * NT;
        int sy = 0, sz = 0;
        if (h < SH::NHALO) halo_pos<R>(h, sy, sz);
        hl[i] = h < SH::NHALO ? (sy + 2 * R) * Z0 + sz + 2 * R : -1;
        hg[i] = ghost(y0 + sy, n1) * pitch + ghost(z0 + sz, n2);
    }

    const int xs = x0 - R;   // first plane of level n+1
    const int xe = x1 + R;   // one past the last
    // u^n queues: q[d] = u^n(xl - R + d), starting at xl = xs
    T qt[2 * R + 1], qs[2 * R + 1], qd[2 * R + 1];
#pragma unroll
    for (int d = 0; d < 2 * R + 1; ++d) {
        const int64_t xo = (int64_t)ghost(xs - R + d, n0) * ps;
        qt[d] = ucur[xo + off_t];
        qs[d] = has_s ? ucur[xo + off_s] : (T)0;
        qd[d] = has_d ? ucur[xo + off_d] : (T)0;
    }
    // u^{n+1} queue of the tile cell (planes xl - 2R - 1 .. xl - 1 at the top of an
    // iteration), the last R ring values of u^{n+1}, and the tile's c over R + 1 planes
    T w1[2 * R + 1], ls[R], ld[R], cq[R + 1];
#pragma unroll
    for (int d = 0; d < 2 * R + 1; ++d) w1[d] = (T)0;
#pragma unroll
    for (int d = 0; d < R; ++d) { ls[d] = (T)0; ld[d] = (T)0; }
#pragma unroll
    for (int d = 0; d < R + 1; ++d) cq[d] = (T)0;

    // plane-xl operands, loaded one plane ahead
    T um_t, um_s, um_d, c_t, c_s, c_d, ch[NH];
    AT ca = (AT)0;
    float cp = 0.f;
    {
        const int64_t xo = (int64_t)ghost(xs, n0) * ps;
        um_t = uprev[xo + off_t];
        um_s = has_s ? uprev[xo + off_s] : (T)0;
        um_d = has_d ? uprev[xo + off_d] : (T)0;
        c_t = cc[xo + off_t];
        c_s = has_s ? cc[xo + off_s] : (T)0;
        c_d = has_d ? cc[xo + off_d] : (T)0;
#pragma unroll
        for (int i = 0; i < NH; ++i) ch[i] = hl[i] >= 0 ? ucur[xo + hg[i]] : (T)0;
    }

    // event walks: ring events of level n+1 at xl; tile events at x2 for the sampling
    // of level n+1 (rows of the first step) and for level n+2 (rows of the second)
    StepArgs aa = a;
    aa.blk_off = p.blk_off_a;
    aa.grp = p.grp_a;
    aa.ev = p.ev_a;
    StepArgs a2 = a;
    a2.row_src = p.row_src2;
    a2.row_rec = p.row_rec2;
    PlaneEvents pa, pb1, pb2;
    events_begin(pa, aa, b);
    events_begin(pb1, a, b);
    events_begin(pb2, a2, b);

    for (int xl = xs; xl < xe; ++xl) {
        const int x2 = xl - R;
        const bool lvl2 = x2 >= x0;
        const bool more = xl + 1 < xe;
        // issue the loads of plane xl + 1 (level n+1) and of x2 + 1 (level n+2)
        T nq_t = (T)0, nq_s = (T)0, nq_d = (T)0, num_t = (T)0, num_s = (T)0, num_d = (T)0;
        T nc_t = (T)0, nc_s = (T)0, nc_d = (T)0, nh[NH];
        AT na = (AT)0;
        float npt = 0.f;
#pragma unroll
        for (int i = 0; i < NH; ++i) nh[i] = (T)0;
        if (more) {
            const int64_t xq = (int64_t)ghost(xl + 1 + R, n0) * ps;
            const int64_t xn = (int64_t)ghost(xl + 1, n0) * ps;
            nq_t = ucur[xq + off_t];
            if (has_s) nq_s = ucur[xq + off_s];
            if (has_d) nq_d = ucur[xq + off_d];
            num_t = __builtin_nontemporal_load(uprev + xn + off_t);
            if (has_s) num_s = uprev[xn + off_s];
            if (has_d) num_d = uprev[xn + off_d];
            nc_t = cc[xn + off_t];
            if (has_s) nc_s = cc[xn + off_s];
            if (has_d) nc_d = cc[xn + off_d];
#pragma unroll
            for (int i = 0; i < NH; ++i)
                if (hl[i] >= 0) nh[i] = ucur[xn + hg[i]];
        }
        const bool lvl2_next = x2 + 1 >= x0 && x2 + 1 < x1;
        if (lvl2_next && live) {
            const int64_t xa = (int64_t)(x2 + 1) * ps + off_t;
            if (rd_acc) na = __builtin_nontemporal_load(acc + xa);
            if (rd_part) npt = __builtin_nontemporal_load(part + xa);
        }

        // stage u^n(xl), the ring's u^{n+1}(x2) and the events
        T* L0 = lds0[xl & 1];
        L0[l0_t] = qt[R];
        if (has_s) L0[l0_s] = qs[R];
        if (has_d) L0[l0_d] = qd[R];
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (hl[i] >= 0) L0[hl[i]] = ch[i];
        T* L1 = lds1[x2 & 1];
        if (lvl2) {
            L1[l1_t] = w1[R + 1];
            if (has_s) L1[l1_s] = ls[0];
            if (has_d) L1[l1_d] = ld[0];
        }
        events_at_plane<T, NT>(pa, aa, est_a, xl, tid);
        if (lvl2) {
            events_at_plane<T, NT>(pb1, a, est_b1, x2, tid);
            events_at_plane<T, NT>(pb2, a2, est_b2, x2, tid);
        }
        __syncthreads();

        // level n+1 at xl: tile cell, ring cell above/below, ring cell left/right
        auto level1 = [&](const T* q, T um, T cv, int l0, int lane) -> T {
            const T u0 = q[R];
            T lap = (T)0;
#pragma unroll
            for (int j = 1; j <= R; ++j) lap += w[j - 1] * ((q[R + j] - u0) + (q[R - j] - u0));
#pragma unroll
            for (int j = 1; j <= R; ++j) lap += w[j - 1] * ((L0[l0 + j * Z0] - u0) + (L0[l0 - j * Z0] - u0));
#pragma unroll
            for (int j = 1; j <= R; ++j) lap += w[j - 1] * ((L0[l0 + j] - u0) + (L0[l0 - j] - u0));
            if (pa.has) lap += point_force<false>(pa, aa, est_a, lane, 0);
            const T coef = a.coef_direct ? cv : dt2 * cv * cv;
            return (u0 + u0) - um + coef * lap;
        };
        const T v_t = level1(qt, um_t, c_t, l0_t, lane_t);
        const T v_s = has_s ? level1(qs, um_s, c_s, l0_s, lane_s) : (T)0;
        const T v_d = has_d ? level1(qd, um_d, c_d, l0_d, lane_d) : (T)0;
        if (live && xl >= x0 && xl < x1) __builtin_nontemporal_store(v_t, out1 + (int64_t)xl * ps + off_t);
#pragma unroll
        for (int d = 0; d < 2 * R; ++d) w1[d] = w1[d + 1];
        w1[2 * R] = v_t;
#pragma unroll
        for (int d = 0; d < R + 1 - 1; ++d) cq[d] = cq[d + 1];
        cq[R] = c_t;

        // level n+2 at x2 on the tile
        if (lvl2) {
            const T u1 = w1[R];   // u^{n+1}(x2)
            T lap = (T)0;
#pragma unroll
            for (int j = 1; j <= R; ++j) lap += w[j - 1] * ((w1[R + j] - u1) + (w1[R - j] - u1));
#pragma unroll
            for (int j = 1; j <= R; ++j) lap += w[j - 1] * ((L1[l1_t + j * Z1] - u1) + (L1[l1_t - j * Z1] - u1));
#pragma unroll
            for (int j = 1; j <= R; ++j) lap += w[j - 1] * ((L1[l1_t + j] - u1) + (L1[l1_t - j] - u1));
            if (pb2.has) lap += point_force<false>(pb2, a2, est_b2, lane_t, 0);
            const T cv = cq[0];
            const T coef = a.coef_direct ? cv : dt2 * cv * cv;
            const T u0 = qt[0];   // u^n(x2)
            const T v2 = (u1 + u1) - u0 + coef * lap;
            if (live) {
                if (a.sample && pb1.has) sample_receivers<false>(pb1, a, est_b1, lane_t, 0, u1);
                if (a.sample && pb2.has) sample_receivers<false>(pb2, a2, est_b2, lane_t, 0, v2);
                const int64_t xo2 = (int64_t)x2 * ps + off_t;
                __builtin_nontemporal_store(v2, out2 + xo2);
                if (terms) {
                    // the interval n, n+1 and, with terms 3, the interval n+1, n+2, in the
                    // order of the one-step launches (own interval first)
                    const AT d1 = (AT)(u1 - u0);
                    const AT d2 = (AT)(v2 - u1);
                    const AT dsum = terms == 3 ? fma(d2, d2, d1 * d1) : fma(d1, d1, (AT)0);
                    const AT tot = rd_part ? dsum + (AT)cp : dsum;
                    if (rd_acc) __builtin_nontemporal_store(a.acc_sign > 0 ? ca + tot : ca - tot, acc + xo2);
                    if (wr_part) __builtin_nontemporal_store((float)tot, part + xo2);
                }
            }
        }

        // rotate to plane xl + 1
        if (more) {
#pragma unroll
            for (int d = 0; d < 2 * R; ++d) { qt[d] = qt[d + 1]; qs[d] = qs[d + 1]; qd[d] = qd[d + 1]; }
            qt[2 * R] = nq_t;
            qs[2 * R] = nq_s;
            qd[2 * R] = nq_d;
#pragma unroll
            for (int d = 0; d < R - 1; ++d) { ls[d] = ls[d + 1]; ld[d] = ld[d + 1]; }
            ls[R - 1] = v_s;
            ld[R - 1] = v_d;
            um_t = num_t; um_s = num_s; um_d = num_d;
            c_t = nc_t; c_s = nc_s; c_d = nc_d;
#pragma unroll
            for (int i = 0; i < NH; ++i) ch[i] = nh[i];
            ca = na;
            cp = npt;
        }
    }
}

template <int R, typename T, typename AT>
static hipError_t launch_pair_t(int nblk, const PairArgs& p, hipStream_t s)
{
    const int grid = ((nblk + 7) / 8) * 8;
    if (p.terms != 0)
        hipLaunchKernelGGL((pair_kernel<R, T, AT, true>), dim3(grid), dim3(PairShape<R>::NT), 0, s, p);
    else
        hipLaunchKernelGGL((pair_kernel<R, T, AT, false>), dim3(grid), dim3(PairShape<R>::NT), 0, s, p);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_pair_r(int dtype, int acc_dtype, int nblk, const PairArgs& p, hipStream_t s)
{
    if (dtype == 1) return launch_pair_t<R, double, double>(nblk, p, s);
    if (acc_dtype == 1) return launch_pair_t<R, float, double>(nblk, p, s);
    return launch_pair_t<R, float, float>(nblk, p, s);
}

hipError_t launch_pair(int r, int dtype, int acc_dtype, int nblk, const PairArgs& p, hipStream_t s)
{
    switch (r) {
    case 1: return launch_pair_r<1>(dtype, acc_dtype, nblk, p, s);
    case 2: return launch_pair_r<2>(dtype, acc_dtype, nblk, p, s);
    case 4: return launch_pair_r<4>(dtype, acc_dtype, nblk, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace fdw
