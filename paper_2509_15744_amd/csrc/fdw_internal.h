// Internal interfaces between the fdwave host runtime and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

// A source or receiver point inside one block's region, sorted by plane.
struct Event {
    int32_t plane;  // coordinate along the marching axis (axis 0)
    int32_t lane;   // position inside the block tile: ly * WZ + lz
    int32_t kind;   // EV_SRC or EV_REC, plus (shot slot << 1)
    int32_t idx;    // source or receiver number
};
enum { EV_SRC = 0, EV_REC = 1 };

// The events of one block in one plane: ev[begin, end).  A block's groups are sorted
// by plane, so the kernel reads one group per plane that has events.
struct EvPlane {
    int32_t plane, begin, end, pad;
};

// Events of one plane of one block that the kernel stages in LDS at once (planes with
// more take a slower path that reads them from global memory one by one).
constexpr int kStagedEvents = 128;
__host__ __device__ inline int ev_kind(int k) { return k & 1; }
__host__ __device__ inline int ev_shot(int k) { return k >> 1; }

// Arguments of one leapfrog step over the whole grid of one problem.  A step
// advances the shots [shot0, shot0 + S) of the problem together (S is the
// kernel's shot count); their wavefields lie shot_stride elements apart.
struct StepArgs {
    const void* ucur;    // level n (backward: j), first shot of the group
    void* unew;          // level n-1 on entry, n+1 on return (backward: j+1 -> j-1)
    const void* c;       // wave speed, or dt^2 c^2 itself when coef_direct; for the
                         // variable-material step the mass coefficient m
    void* acc;           // sensitivity accumulator shared by the shots (acc_sign != 0)
    const void* stiff;   // variable-material step: stiffness coefficient b per cell
    void* acc_b;         // variable-material step: stiffness-term accumulator
    int64_t shot_stride; // elements between the wavefields of consecutive shots
    int32_t n0, n1, n2;  // extents; 2D grids run with n1 = 1
    int32_t pitch;       // elements between consecutive rows (>= n2; the variable-material
                         // step pads rows to 256-byte alignment, the others use n2)
    double w[8];         // a_j / dx^2, j = 1..r
    double dt2;          // dt^2
    int32_t coef_direct; // 1: c already holds dt^2 c^2
    int32_t acc_sign;    // 0: no accumulation, +1: acc += sum_s d_s^2, -1: acc -= ...
    int32_t acc_cross;   // 1: the sum is over slot pairs, d_0 d_1 (+ d_2 d_3), not squares
    int32_t acc_prev;    // 1: also add the interval before, d = ucur - unew (on entry)
    int32_t acc_face;    // variable-material step: 0, or the sign of the face terms into acc_b
    int32_t active;      // 0: the problem has no step here (multi-problem launches)
    // Partial sums of the kernel terms (f32 fields with an f64 accumulator): the
    // accumulating launches of a sweep add their terms to a per-cell f32 partial sum
    // and fold it into the f64 accumulator every kPartialCycle-th of them, so most
    // accumulating launches move 8 bytes of partial sum per cell instead of 16 of
    // accumulator.  part_mode says what this launch does (PM_*); part is the buffer.
    void* part;
    int32_t part_mode;
    // the same for the stiffness-term accumulator acc_b of the variable-material step,
    // whose terms every launch adds (cycles of kPartialCycle launches)
    void* part_b;
    int32_t part_b_mode;
    // events
    const int32_t* blk_off;  // [nblk + 1] ranges into grp
    const EvPlane* grp;      // per block, its planes that hold events
    const Event* ev;
    const void* wavelet;     // [nt][nsrc]
    int32_t nsrc;
    int32_t row_src;         // wavelet row injected in this step
    double inv_vol;          // 1 / dx^d
    int32_t sample;          // forward: write traces and residuals at receivers
    int32_t inject_rec;      // backward: inject rec_scale * residual at receivers
    void* traces;            // [nt][nrec] or null
    void* resid;             // [nt][nrec]
    const void* obs;         // [nt][nrec]
    int32_t nrec;
    int32_t row_rec;         // trace row written (forward) or residual row injected (backward)
    double rec_scale;        // -k / dt
    // block decomposition
    int32_t nty, ntz, chunk_len, nblk;
};

// What an accumulating launch does with the kernel terms it computes (dsum):
//   PM_DIRECT  acc += sign dsum                 (no partial sum pending)
//   PM_START   part = dsum
//   PM_ADD     part += dsum
//   PM_FLUSH   acc += sign (part + dsum)
// The partial sum is rounded to f32 when stored; every kPartialCycle-th accumulating
// launch of a sweep folds it into the accumulator, and the last one always does.
enum { PM_DIRECT = 0, PM_START = 1, PM_ADD = 2, PM_FLUSH = 3 };
constexpr int kPartialCycle = 16;

// Tile shape of one kernel variant.
struct Variant {
    int32_t tz;      // tile width in cells along the contiguous axis
    int32_t ty;      // tile height along axis 1 (3D only)
    int32_t threads; // threads per block
    int32_t vz;      // consecutive cells per lane (the contiguous extent must be a multiple)
    int32_t max_shots; // largest shot group the variant is built for (1, 2 or 4)
};

int variant_count(int ndim);
Variant variant_shape(int ndim, int variant);  // variant in 1..count

// One step of one problem for a group of `shots` shots (1, 2 or 4).
hipError_t launch_step(int ndim, int r, int dtype, int acc_dtype, int variant, int shots,
                       int nblk, const StepArgs& a, hipStream_t s);

// One step of the variable-material second-order scheme (one wavefield; tile shapes of
// step variants 1 and 2).  a.c is the mass coefficient, a.stiff the stiffness.
hipError_t launch_vd_step(int ndim, int dtype, int acc_dtype, int variant, int nblk, const StepArgs& a,
                          hipStream_t s);

// Misc kernels.  All return hipError_t of the launch.
hipError_t launch_speed_stats(int dtype, const void* c, int64_t n, double* d_out3, double* d_part,
                              hipStream_t s);
// d_out[0] = scale * sum (x - y)^2 (x^2 when y is null) in fixed order; diff_out (may be
// null) receives x - y.  d_part holds kReduceBlocks doubles.
hipError_t launch_sum_squares(int dtype, const void* x, const void* y, void* diff_out, int64_t n,
                              double* d_part, double* d_out, hipStream_t s, double scale = 1.0);
// Zero `bytes` (a multiple of 4) at p (16-byte aligned) with a kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// Copy `rows` rows of n2 elements of size es (4 or 8) between row strides spitch and dpitch.
hipError_t launch_copy_rows(void* dst, int64_t dpitch, const void* src, int64_t spitch, size_t es,
                            int64_t rows, int64_t n2, hipStream_t s);
// J[0..n) = NaN when *flag != 0 (a persistent launch gave up at a grid barrier).
hipError_t launch_nan_if_flag(const unsigned* flag, double* J, int n, hipStream_t s);
// Terminal hand-over for the shots [shot0, shot0 + nshots) of a problem: per distinct
// receiver cell, receivers sorted by (cell, shot); u_last / u_prev point at the
// group's first shot, shots shot_stride elements apart.  The step coefficient is
// dt2 c^2 from the speed c, or dt2 / c when `mass` (c is then the mass coefficient).
hipError_t launch_terminal(int dtype, int acc_dtype, int nuniq, const int64_t* ucell,
                           const int32_t* uoff, const int32_t* uidx, const int32_t* ushot,
                           int shot0, int nshots, int64_t shot_stride, const void* c, int mass,
                           double dt2, const void* u_last, void* u_prev, void* acc,
                           const void* resid_row, double rec_scale, hipStream_t s);
// Terminal hand-over of the re-simulation sweep for the shots [shot0, shot0 + nshots):
// mu^{nt-1} = coef * fdag^{nt} at the receiver cells of each shot (mu^{nt} = 0) and the
// kernel of the last interval, -(u^nt - u^{nt-1}) mu^{nt-1}.  u_last / u_prev point at
// the first shot's u; shot s's u sits s * shot_stride further and its mu a further
// mu_offset elements on.
hipError_t launch_terminal_exact(int dtype, int acc_dtype, int nuniq, const int64_t* ucell,
                                 const int32_t* uoff, const int32_t* uidx, const int32_t* ushot,
                                 int shot0, int nshots, int64_t shot_stride, int64_t mu_offset,
                                 const void* c, double dt2, const void* u_last, void* u_prev,
                                 void* acc, const void* resid_row, double rec_scale, hipStream_t s);
hipError_t launch_finalize(int dtype, int acc_dtype, int64_t n, const void* acc, const void* c,
                           double scale, void* grad, hipStream_t s);
// out = scale * acc (accumulator dtype to grid dtype).
hipError_t launch_scale(int dtype, int acc_dtype, int64_t n, const void* acc, double scale, void* out,
                        hipStream_t s);

constexpr int kReduceBlocks = 512;
constexpr int kReduceThreads = 256;

}  // namespace fdw
