/*
 * fdwave: memory-efficient adjoint sensitivities of the scalar acoustic wave
 * equation on AMD MI355X (gfx950).
 *
 * Method: Herrmann, Buerchner, Kudela, Kollmannsberger, "A Memory Efficient
 * Adjoint Method to Enable Billion Parameter Optimization on a Single GPU in
 * Dynamic Problems", arXiv:2509.15744.  The sensitivity is the mixed kernel
 * of the superposed field v = u + k u_dagger (Sec. 4, Eq. superposedkernel),
 * computed by Algorithm 1: a forward sweep that accumulates K(u,u), then a
 * backward sweep of the superposed field that accumulates K(v,v), so that no
 * forward history is stored.
 *
 * Physics and discretisation (Sec. 2.3, Eq. wavetopopt with rho^-1 = 1 and
 * kappa = c^2; Sec. 3.1, Eq. FDstencil2 extended to a 2r-th order central
 * Laplacian):
 *
 *     u^{n+1} = 2 u^n - u^{n-1} + dt^2 c^2 (L u^n + f^n)
 *     (L u)_i = dx^-2 sum_axes sum_{j=1..r} a_j [(u_{i+j} - u_i) + (u_{i-j} - u_i)]
 *
 * with homogeneous Neumann walls (Eq. BC) as half-sample mirror ghost cells
 * (Sec. 3.1): a ghost index -1-j reads cell j and n+j reads cell n-1-j.
 *
 * Time axis: u^{-1} = u^0 = 0 (Eq. IC).  Forward steps n = 0..nt-1 produce
 * u^1..u^nt.  The point force of step n is f^n = wavelet[n][s] / dx^d at
 * source cell s (Eq. source1).  Receivers record u^1..u^nt: row n-1 of every
 * [nt][nrec] trace array holds level n.
 *
 * Misfit (Eq. cost1 with the time integral as dt * sum):
 *     J = dt/2 sum_{n=1..nt} sum_r (u^n(x_r) - obs^n_r)^2
 * Gradient: dJ/dc per cell, dJ/dc = -(2/c^3) dJ/dm with m = 1/c^2, and the
 * kernel in m for level sequences a, b is K(a,b) = -sum_n (a^{n+1}-a^n)(b^{n+1}-b^n)
 * (the mass term of Eq. kernel2 in discrete form).  The approximation is
 *     dJ/dm ~ (K(v,v) - K(u,u)) / (2k)
 * and differs from the exact discrete adjoint by k/2 K(mu,mu) (Eq.
 * superposedkernel1).
 *
 * Layouts: every grid array is C-order [n0][n1] or [n0][n1][n2], last axis
 * contiguous, axis 0 the depth axis.  Cells are named by flat C-order int64
 * indices.
 *
 * Ownership: the caller owns every pointer passed in; the library never
 * frees or retains one after a call returns.  Arrays marked DEVICE live in
 * the current HIP device's memory; arrays marked HOST are read during the
 * call only.  Temporary device memory is taken stream-ordered on `stream`
 * and released before the call returns.
 *
 * Streams: all device work is enqueued on `stream` (a hipStream_t; NULL is
 * the null stream).  Calls that return a host value (J, c_max) synchronise
 * that stream before returning.
 *
 * Errors: every entry point returns FD_OK (0) or a positive FD_E_* code and
 * leaves a message for fd_last_error() in the calling thread.  Outputs are
 * unspecified after an error.  No C++ exception crosses this interface.
 */
#ifndef FDWAVE_H
#define FDWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FD_OK 0
#define FD_E_ARG 1        /* null pointer, bad ndim/order/dtype, shape < r, index out of range, nt < 1, k = 0 ... */
#define FD_E_CFL 2        /* c_max dt / dx above the leapfrog stability limit */
#define FD_E_NOMEM 3      /* device allocation failed */
#define FD_E_DEVICE 4     /* a HIP call failed; fd_last_error() carries its text */
#define FD_E_NONFINITE 5  /* non-finite or non-positive speed, or a non-finite result */

#define FD_F32 0
#define FD_F64 1

typedef struct fd_grid {
    int32_t ndim;       /* 2 or 3 */
    int64_t shape[3];   /* extents n0, n1[, n2]; each >= order/2; shape[2] ignored when ndim = 2 */
    double dx;          /* cell size, > 0, the same on every axis */
    int32_t order;      /* space order: 2, 4 or 8 */
    int32_t dtype;      /* FD_F32 or FD_F64: element type of every field, wavelet and trace array */
} fd_grid;

/* Acquisition of one problem.  A batch of shots on the same medium is one acquisition
 * whose sources and receivers carry shot numbers: each shot is its own wave field
 * (driven by its own sources, recorded by its own receivers), J sums over all
 * receivers and the gradient over all shots (one shared accumulator).  With nshot
 * 0 or 1 there is one shot and the tag arrays are ignored. */
typedef struct fd_acq {
    int32_t nsrc;             /* number of point sources, >= 0 */
    const int64_t* src_cell;  /* HOST [nsrc] flat cell of each source (repeats allowed) */
    const void* wavelet;      /* DEVICE [nt][nsrc] source time functions, row n at t = n dt */
    int32_t nrec;             /* number of receivers, >= 0 */
    const int64_t* rec_cell;  /* HOST [nrec] flat cell of each receiver (repeats allowed) */
    int32_t nshot;            /* number of shots (0 or 1: a single shot) */
    const int32_t* src_shot;  /* HOST [nsrc] shot of each source, in [0, nshot) */
    const int32_t* rec_shot;  /* HOST [nrec] shot of each receiver, in [0, nshot) */
} fd_acq;

/* Optional timing record, filled by a call whose fd_opts.timing points here: HIP events
 * on `stream` bracket the step launches of each sweep (one step kernel per time step). */
typedef struct fd_timing {
    double fwd_ms;          /* device time from the first to the last forward step launch */
    int32_t fwd_launches;   /* forward step launches in that interval */
    double bwd_ms;          /* the same for the backward sweep (superposed or re-simulation) */
    int32_t bwd_launches;
    int32_t fwd_pair_launches;  /* of the launches: those that advanced two steps (fd_opts.pairs) */
    int32_t bwd_pair_launches;
    int32_t persistent_blocks;  /* batch plans with persistent launches: blocks that took part in
                                   the last sweep (fd_batch_timing; 0 otherwise) */
} fd_timing;

typedef struct fd_opts {
    int32_t acc_dtype;  /* sensitivity accumulator: FD_F64 (default) or FD_F32 (f32 grids only) */
    int32_t variant;    /* kernel tile variant; 0 lets the library choose (see fd_variant_count) */
    fd_timing* timing;  /* HOST, may be NULL: when set, the call also synchronises `stream` */
    int32_t chunk;      /* planes of axis 0 marched per block; 0 lets the library choose */
    int32_t max_group;  /* shots advanced per launch: 1, 2 or 4 (0: the largest the variant has) */
    int32_t graph;      /* batched calls: 1 replays each sweep as one captured hipGraph */
    int32_t persistent; /* batched calls: 1 runs each sweep as one launch whose running blocks
                           (counted at run time) each own one group (a column of consecutive
                           chunks, sized so the groups do not outnumber them; a block may
                           own several when even whole columns do) and walk all steps, a
                           group starting a step once its neighbouring groups have finished
                           the previous one */
    int32_t barrier_timeout_us; /* persistent launches: longest wait of a group for its
                           neighbours before the launch gives up and the call returns
                           FD_E_DEVICE (0: 2 s) */
    int32_t variant_plain; /* tile variant of the step launches that do not touch the
                           accumulator (about half of each sweep); 0: the same as `variant`
                           (or the remembered choice when `variant` is 0).  Used only where
                           it groups the shots as `variant` does; results are identical */
    int32_t chunk_plain;   /* planes per block for those launches; 0: library choice */
    int32_t no_partials;   /* 1: every accumulating step reads and writes the f64
                           accumulator; 0 (default): f32 fields with an f64 accumulator
                           keep f32 partial sums of the kernel terms, folded into the
                           accumulator every 16th accumulating step (4 instead of 8 bytes
                           of accumulator traffic per cell update on average) */
    int32_t pairs;         /* 1: the constant-density 3D sweeps of one shot advance two time
                           steps per launch (levels n+1 and n+2 from n-1 and n; 28 instead
                           of 40 bytes per cell for two steps with partial sums; results
                           equal those of one step per launch) where every extent is at
                           least the order; 0: library choice (one step per launch);
                           -1: never.  Takes two more wavefields of scratch */
} fd_opts;

/* Caller-owned device state that carries one gradient from its forward sweep
 * (fd_sens_forward) to its backward sweep (fd_sens_backward). */
typedef struct fd_state {
    void* u_a;       /* DEVICE [nshot][ncell] grid dtype */
    void* u_b;       /* DEVICE [nshot][ncell] grid dtype */
    void* acc;       /* DEVICE [ncell] accumulator dtype: K(u,u) - K(v,v) in progress */
    void* residual;  /* DEVICE [nt][nrec] grid dtype: u^n(x_r) - obs^n_r */
} fd_state;

/* One independent problem of a batched call (its own medium, grid, acquisition, time
 * axis and k).  All problems of one call share ndim, order and dtype. */
typedef struct fd_problem {
    fd_grid grid;
    const void* c;          /* DEVICE [ncell] wave speed */
    fd_acq acq;             /* single shot (nshot 0 or 1) */
    double dt;
    int32_t nt;
    const void* observed;   /* DEVICE [nt][nrec] */
    double k;
    void* grad_c;           /* DEVICE [ncell] output dJ/dc */
    void* traces;           /* DEVICE [nt][nrec] output, or NULL */
} fd_problem;

/* Message of the last failed call in this thread ("" if none). */
const char* fd_last_error(void);

/* Largest stable Courant number c_max dt / dx for the leapfrog with the order-`order`
 * central stencil in `ndim` dimensions (2 / sqrt(ndim * |symbol(pi)|)); 0 if invalid. */
double fd_cfl_limit(int32_t ndim, int32_t order);

/* Upper bound of the device memory one fd_adjoint_sensitivity call on this grid and
 * acquisition takes from the stream-ordered pool of `stream`'s device, beyond the
 * caller's inputs and outputs (host-side arithmetic, no device work):
 *   wavefields 2 * nshots * ncell * sizeof(T), accumulator ncell * 8 (f64, the larger
 *   choice), for f32 grids ncell * 4 of f32 partial sums of the kernel terms (which an
 *   f64 accumulator takes in every 16th accumulating step), residual rows
 *   nt * nrec * sizeof(T) — with ncell counted in rows padded to
 *   64 elements when the contiguous extent is not a multiple of 64, plus then a padded
 *   copy of c and a padded finalisation buffer — event tables of two launch plans
 *   (per-block offsets for every shot group, bounded with the smallest tile and one
 *   plane per block) and the reduction partials.  acq may be NULL (no sources or receivers); nshots < 1 counts as 1.
 * Returns 0 and sets fd_last_error on an invalid grid or a negative nt.  The split
 * halves take the same amount less the caller-owned fd_state arrays (plus padded
 * working copies of those arrays when rows are padded). */
size_t fd_workspace_bytes(const fd_grid* grid, const fd_acq* acq, int32_t nt, int32_t nshots);

/* Number of kernel tile variants for `ndim` (valid fd_opts.variant values are 1..count). */
int32_t fd_variant_count(int32_t ndim);

/* Shape of tile variant `variant` (1..count) for `ndim`: tile width along the contiguous
 * axis and height along axis 1 in cells, threads per block, cells per lane along the
 * contiguous axis (a variant runs only on grids whose contiguous extent is a multiple of
 * it), and the most wavefields one launch advances together (shots of a group, or the
 * two fields of the exact re-simulation).  Any output pointer may be NULL.  Returns
 * FD_OK or FD_E_ARG. */
int fd_variant_info(int32_t ndim, int32_t variant, int32_t* tile_z, int32_t* tile_y,
                    int32_t* threads, int32_t* cells_per_lane, int32_t* max_fields);

/* Autotuner: times `steps` fused steps of each kind the sweeps alternate (adding two
 * kernel terms; touching no accumulator) for every tile variant that fits the grid,
 * several axis-0 chunk lengths and, for nshot > 1, the shot-group sizes, on scratch
 * fields of this grid allocated and freed by the call; writes the fastest shape of each
 * kind for the best shot-group size (time per shot-cell update of the pair) into *best
 * (variant, chunk, max_group, variant_plain, chunk_plain; other fields copied from
 * opts) and remembers it for this process under the key (GPU architecture, HIP
 * runtime version, ndim, order, dtype, accumulator dtype, shape, shot count).  Calls
 * whose fd_opts.variant is 0 use a remembered entry of their key (their chunk and
 * max_group too, unless set).  If the environment variable FDWAVE_TUNE_CACHE names a
 * file, entries are appended to it as JSON lines and read back on first use.
 * best_ms (may be NULL) receives the best time per step.  Synchronises `stream`. */
int fd_autotune(const fd_grid* grid, int32_t nshot, const fd_opts* opts, int32_t steps,
                fd_opts* best, double* best_ms, void* stream);

/* Forward solve (Alg. 1 forward loop without cost or kernel): traces DEVICE [nt][nrec]
 * receive u^1..u^nt at the receivers.  c DEVICE [ncell] is the wave speed. */
int fd_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int32_t nt,
               void* traces, const fd_opts* opts, void* stream);

/* Misfit J = dt/2 sum (traces - observed)^2 (Eq. cost1) over [nt][nrec] DEVICE arrays of
 * `dtype`; residual_or_null DEVICE [nt][nrec] receives traces - observed; J_host receives J
 * (reduced in fixed order in double precision). */
int fd_misfit(int32_t nt, int32_t nrec, int32_t dtype, double dt, const void* traces,
              const void* observed, void* residual_or_null, double* J_host, void* stream);

/* Memory-efficient sensitivity (Alg. 1): J and grad_c DEVICE [ncell] = dJ/dc at factor k
 * (k != 0, finite; the same k gives the same result on every call).  observed DEVICE
 * [nt][nrec]; traces_or_null DEVICE [nt][nrec]. */
int fd_adjoint_sensitivity(const fd_grid* grid, const void* c, const fd_acq* acq, double dt,
                           int32_t nt, const void* observed, double k, void* grad_c,
                           double* J_host, void* traces_or_null, const fd_opts* opts,
                           void* stream);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): fd_adjoint_sensitivity with the same
 * arguments and results, whose scratch (wavefields, accumulator, partial sums,
 * residual rows, padded copies, event tables, reduction partials) is carved out of a
 * fixed device array of FD_NOALLOC_BYTES that every GPU the library runs on holds
 * from the library's load until the process ends.  The call performs no device
 * allocation or release.  A problem whose scratch bound exceeds the array returns
 * FD_E_ARG with the two sizes in fd_last_error() before any device work.  The array
 * keeps the last call's contents; the call clears what must start at zero.  Calls on
 * one GPU share its array: the library serialises them (a per-device lock held until
 * the call's work on `stream` has finished), so this call always synchronises
 * `stream`; the current device must be `stream`'s device. */
#define FD_NOALLOC_BYTES ((size_t)64 << 20)
int fd_adjoint_sensitivity_noalloc(const fd_grid* grid, const void* c, const fd_acq* acq, double dt,
                                   int32_t nt, const void* observed, double k, void* grad_c,
                                   double* J_host, void* traces_or_null, const fd_opts* opts,
                                   void* stream);

/* Exact discrete gradient by re-simulation (the alternative to the superposition that the
 * paper's introduction cites; no stored history, no factor k): a forward sweep with cost
 * and adjoint force but no kernel accumulation, then one backward sweep that steps u
 * back from (u^nt, u^{nt-1}) with the same scheme together with the adjoint field mu
 * (mu^nt = 0, mu^{nt-1} = dt^2 c^2 fdag^nt at the receivers, fdag^n = -(u^n(x_r) -
 * observed^n_r)/dt) and accumulates sum_n (u^{n+1} - u^n)(mu^{n+1} - mu^n) per cell;
 * grad_c DEVICE [ncell] = 2 acc / c^3 = dJ/dc of the discrete J, exact up to rounding
 * (the re-simulated u carries the rounding of the backward recursion).  Arguments as for
 * fd_adjoint_sensitivity without k; every shot is one two-field launch per step, so
 * fd_opts.variant must carry two fields (variants 1 and 2; 0 picks one) and
 * fd_opts.max_group is ignored.  Scratch: four wavefields per shot, the accumulator and
 * the residuals, allocated stream-ordered and freed by the call.  Synchronises `stream`. */
int fd_adjoint_exact(const fd_grid* grid, const void* c, const fd_acq* acq, double dt, int32_t nt,
                     const void* observed, void* grad_c, double* J_host, void* traces_or_null,
                     const fd_opts* opts, void* stream);

/* The paper's own second-order flux-form scheme with variable material (Sec. 3.1,
 * Eqs. FDstencil1/FDstencil2), written as m u_tt - div(b grad u) = f with a mass
 * coefficient m and a stiffness coefficient b per cell (rho-scaling, Eq.
 * scalarwaveequation: m = gamma rho0, b = gamma rho0 c0^2; Eq. wavetopopt: m = 1/kappa,
 * b = 1/rho):
 *     u^{n+1} = 2 u^n - u^{n-1} + (dt^2 / m) (L_b u^n + f^n)
 *     (L_b u)_i = dx^-2 sum over the 2d neighbours j:  h(b_i, b_j) (u_j - u_i),
 *     h(p, q) = 2 p q / (p + q)  (harmonic mean at the face)
 * Wall ghosts mirror the boundary cell and carry its material (no flux through a wall).
 * grid->order must be 2.  m, b DEVICE [ncell], finite and positive; dt must satisfy
 * dt^2 max_i s_i <= 4 dx^2 (else FD_E_CFL), s_i = sum over the interior faces of cell i
 * of h_f (1/m_i + 1/sqrt(m_i m_j)): the Gershgorin bound of the leapfrog limit
 * dt^2 lambda_max(M^-1 K) < 4, equal to dt sqrt(d b/m) <= dx in a homogeneous medium
 * and local where materials mix.  When the contiguous extent is not a multiple of
 * 64 the sweeps run on copies with rows padded to 64 elements (m and b, the
 * wavefields and both accumulators; stream-ordered scratch of up to about six grid
 * arrays beyond the unpadded case), which keeps every row load on 256-byte
 * boundaries; callers' arrays stay dense.  Time axis, sources, receivers, shots
 * and misfit as for the constant-density calls.  fd_opts.variant: 0, 1, 2 or 5 (3D also 7, 2D also 4);
 * max_group is ignored (one wavefield per launch). */
int fd_vd_forward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt,
                  int32_t nt, void* traces, const fd_opts* opts, void* stream);

/* Alg. 1 for the variable-material scheme at factor k: J and the sensitivities
 * grad_m = dJ/dm and grad_b = dJ/db, DEVICE [ncell] each, the two terms of the paper's
 * kernel (Eqs. kernel1/kernel2) in discrete form.  The forward sweep accumulates
 * K_m(u,u) = sum_n (u^{n+1} - u^n)^2 and K_b(u,u) = sum_n sum_faces dh/db_i
 * (u_j^n - u_i^n)^2, the superposed backward sweep the same of v = u + k mu; then
 *     grad_m = (K_m(u,u) - K_m(v,v)) / (2k),
 *     grad_b = -(dt^2 / dx^2) (K_b(u,u) - K_b(v,v)) / (2k),
 * which differ from the exact discrete gradient by -(k/2) sum_n (mu^{n+1} - mu^n)^2 and
 * (dt^2/dx^2)(k/2) sum_n sum_faces dh/db_i (mu_j^n - mu_i^n)^2.  A gradient with respect
 * to a design field gamma follows by the chain rule (e.g. rho-scaling: rho0 grad_m +
 * rho0 c0^2 grad_b).  Scratch: two wavefields per shot, two accumulators and the
 * residuals, allocated stream-ordered and freed by the call.  Synchronises `stream`. */
int fd_vd_adjoint_sensitivity(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq,
                              double dt, int32_t nt, const void* observed, double k, void* grad_m,
                              void* grad_b, double* J_host, void* traces_or_null, const fd_opts* opts,
                              void* stream);

/* The two halves of fd_vd_adjoint_sensitivity with caller-owned state (as for the
 * constant-density split below): `state` holds the wavefields, the mass-term
 * accumulator and the residuals, `acc_b` DEVICE [ncell] (accumulator dtype) the
 * stiffness-term accumulator.  The forward half leaves u^{nt-1}, u^nt, both
 * accumulators and the residuals; the backward half consumes them and writes
 * grad_m = grad_scale dJ/dm and grad_b = grad_scale dJ/db.  Same grid, m, b, acq, dt, nt
 * and opts in both calls. */
int fd_vd_sens_forward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt,
                       int32_t nt, const void* observed, const fd_state* state, void* acc_b,
                       void* traces_or_null, double* J_host, const fd_opts* opts, void* stream);
int fd_vd_sens_backward(const fd_grid* grid, const void* m, const void* b, const fd_acq* acq, double dt,
                        int32_t nt, double k, const fd_state* state, void* acc_b, double grad_scale,
                        void* grad_m, void* grad_b, const fd_opts* opts, void* stream);

/* First half of fd_adjoint_sensitivity: the forward sweep with cost, adjoint force and
 * K(u,u) accumulation; leaves u^{nt-1}, u^nt, the accumulator and the residuals in
 * `state` (all four arrays overwritten).  J_host may be NULL.  When the contiguous
 * extent is not a multiple of 64 this call, its second half, fd_forward and
 * fd_adjoint_sensitivity sweep on copies with rows padded to 64 elements (256-byte
 * aligned row loads); `state` stays in the caller's dense layout. */
int fd_sens_forward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt,
                    int32_t nt, const void* observed, const fd_state* state,
                    void* traces_or_null, double* J_host, const fd_opts* opts, void* stream);

/* Second half: the superposed backward sweep from `state` (consumed: its arrays are
 * overwritten) and grad_c = grad_scale * dJ/dc.  Same grid, c, acq, dt, nt and opts
 * as the fd_sens_forward call that filled `state`. */
int fd_sens_backward(const fd_grid* grid, const void* c, const fd_acq* acq, double dt,
                     int32_t nt, double k, const fd_state* state, double grad_scale,
                     void* grad_c, const fd_opts* opts, void* stream);

/* Alg. 1 for `nprob` independent problems of uneven sizes in lock-step: every time
 * step of all problems is one launch over the union of their tiles (problems that
 * have no step there skip it), the backward sweeps are aligned at their ends.  With
 * opts->persistent each sweep is one launch whose blocks walk all its steps (a group
 * of chunks waits for its neighbouring groups' previous step, not for the whole
 * grid).  This is a batch plan (below) created, run once and destroyed: with
 * opts->graph the run is captured into a hipGraph and launched as one graph.  J_host
 * [nprob] receives each problem's J; synchronises `stream`.  Needs opts variant 0, 1
 * or 2 (2D also 4 and 5).  FD_E_DEVICE if a persistent launch's wait for the
 * launch's other blocks or for neighbouring groups timed out. */
int fd_adjoint_sensitivity_batched(const fd_problem* probs, int32_t nprob, double* J_host,
                                   const fd_opts* opts, void* stream);

/* The batched call as a reusable plan whose run is graph-capturable (Alg. 1 per
 * problem, as above).  The paper states the time per time step per source (Tab.
 * timings); a plan amortises everything that needs the host across runs: a run
 * issues kernel launches only.
 *
 * fd_batch_plan_create validates the problems (as fd_adjoint_sensitivity_batched),
 * checks every speed field against the CFL limit once, builds the block
 * decompositions, event tables and step-argument tables, allocates the state of
 * every problem (two wavefields, the accumulator, the residual rows; rows padded to
 * 64 elements where the contiguous extent needs it) stream-ordered on `stream`, and
 * synchronises `stream` once.  *plan receives the plan (NULL on error).  The plan
 * keeps the device pointers of every problem (c, wavelet, observed, grad_c, traces):
 * they must stay valid, at the same addresses, until the plan is destroyed.  The host
 * arrays of the acquisitions (cells, shot tags) are read during this call only.
 * fd_opts: variant 0, 1 or 2, acc_dtype, persistent, barrier_timeout_us, timing (a
 * run then records HIP events around both sweeps; read them with fd_batch_timing);
 * graph is ignored (the caller captures runs itself).
 *
 * fd_batch_run enqueues one gradient of every problem on `stream`: state zeroed by
 * kernels, each problem's current c copied into the padded layout where needed, the
 * forward sweeps, the terminal hand-overs, the backward sweeps, grad_c, and
 * J DEVICE [nprob] doubles (J[p] = dt_p/2 sum of problem p's squared residuals,
 * reduced in fixed order).  It allocates nothing, copies nothing to or from the host,
 * records no memset and does not synchronise, so a stream capture of it is a graph
 * that may be replayed: each replay reads the values c, wavelet and observed hold
 * then.  The CFL check of fd_batch_plan_create is not repeated: a c that has become
 * unstable since gives non-finite values.  With opts.persistent every J of the run
 * is NaN if a wait for neighbouring groups timed out.  Runs of one plan share its state: they
 * must not overlap (one stream, or ordered by the caller).  FD_E_ARG for a null plan
 * or J; a failed launch gives FD_E_DEVICE.
 *
 * fd_batch_timing waits for the last run's second sweep and fills *timing with the
 * device time of its two sweeps (FD_E_ARG if the plan was made without timing).
 *
 * fd_batch_plan_destroy releases the plan's device memory stream-ordered on `stream`
 * (no run of it may be pending on another stream) and the plan itself; NULL is a
 * no-op. */
typedef struct fd_batch_plan fd_batch_plan;
int fd_batch_plan_create(const fd_problem* probs, int32_t nprob, const fd_opts* opts, void* stream,
                         fd_batch_plan** plan);
int fd_batch_run(fd_batch_plan* plan, double* J, void* stream);
int fd_batch_timing(fd_batch_plan* plan, fd_timing* timing);
int fd_batch_plan_destroy(fd_batch_plan* plan, void* stream);

/* Source-free steps (test hook for closed-form solutions): on entry u_prev, u_cur DEVICE
 * [ncell] hold levels -1 and 0; on return they hold levels nsteps-1 and nsteps.
 * coef DEVICE [ncell] is dt^2 c^2 itself (no CFL check). */
int fd_propagate(const fd_grid* grid, const void* coef, void* u_prev, void* u_cur,
                 int32_t nsteps, const fd_opts* opts, void* stream);

/* ---- gradient-based design around the sweeps ------------------------------------
 * A design field gamma lives on a box of cells inside the grid (one value per box
 * cell, C order over the box).  The material of the variable-material calls is made
 * from it by the topology-optimisation chain of Sec. 2.3 (Constraints):
 *   filtered   gt_i = sum_k w_ik gamma_k / sum_k w_ik,  w_ik = r_f - |x_i - x_k| for
 *              |x_i - x_k| < r_f (in cells), k over the box (density filter with
 *              linear decay);
 *   projected  h_i = (tanh(beta eta) + tanh(beta (gt_i - eta)))
 *                    / (tanh(beta eta) + tanh(beta (1 - eta)))   (smoothed Heaviside);
 *   clipped    g_i = min(max(h_i, lo), hi);
 *   material   m = m0 + g dm,  b = b0 + g db   at the grid cell of box cell i.
 * Both of the paper's maps are this affine form: rho-scaling (Eq.
 * scalarwaveequation) m0 = b0 = 0, dm = rho0, db = rho0 c0^2; the two-material map
 * (Eq. wavetopopt) m0 = 1/kappa1, dm = 1/kappa2 - 1/kappa1, b0 = 1/rho1,
 * db = 1/rho2 - 1/rho1.  Grid cells outside the box keep their values. */
typedef struct fd_design {
    int32_t ndim;          /* 2 or 3 */
    int64_t shape[3];      /* grid extents (m, b and their gradients are [shape], C order) */
    int64_t origin[3];     /* first grid cell of the box, per axis */
    int64_t extent[3];     /* box extents (>= 1); the box must lie inside the grid */
    int32_t dtype;         /* FD_F32 or FD_F64 for every field of these calls */
    double filter_radius;  /* r_f in cells, at most 32; r_f <= 1 means no filter */
    double beta, eta;      /* projection sharpness (> 0) and threshold in [0, 1]; beta <= 0: none */
    double lo, hi;         /* clip interval of the projected field, lo <= hi */
    double m0, dm, b0, db; /* affine material map (finite) */
} fd_design;

/* Material from the design field: writes m and b DEVICE [shape] at the box cells and,
 * when gamma_bar is not NULL, the clipped projected field DEVICE [box] (the field the
 * material is affine in).  gamma DEVICE [box].  FD_E_ARG on a bad description or null
 * pointers; no synchronisation. */
int fd_design_map(const fd_design* design, const void* gamma, void* m, void* b, void* gamma_bar,
                  void* stream);

/* The chain rule of fd_design_map (Sec. 2.3): from grad_m = dC/dm and grad_b = dC/db
 * (DEVICE [shape]; read at the box cells) to grad_gamma = dC/dgamma DEVICE [box]:
 *   dC/dgamma_k = sum_i w_ik / W_i * [lo <= h_i <= hi] * dh/dgt(gt_i) * (dm grad_m_i + db grad_b_i),
 * W_i = sum_k w_ik, the derivative of the clip taken as 1 on the closed interval and 0
 * outside.  Takes one box-sized scratch buffer (stream-ordered); FD_E_NOMEM if it cannot. */
int fd_design_adjoint(const fd_design* design, const void* gamma, const void* grad_m, const void* grad_b,
                      void* grad_gamma, void* stream);

/* One Adam step (the optimiser the paper pairs with Eq. gradientdescent) on x DEVICE [n]
 * from grad DEVICE [n], with first and second moments m1, m2 DEVICE [n] updated in place
 * (zero before step 1):
 *   m1 = beta1 m1 + (1 - beta1) g,   m2 = beta2 m2 + (1 - beta2) g^2,
 *   x -= lr (m1 / (1 - beta1^step)) / (sqrt(m2 / (1 - beta2^step)) + eps),
 * then x is clipped to [lo, hi] (the paper clips the design field after each update).
 * step >= 1; 0 <= beta1, beta2 < 1; eps >= 0; lr finite; lo <= hi. */
int fd_adam_step(int64_t n, int32_t dtype, void* x, const void* grad, void* m1, void* m2, int32_t step,
                 double lr, double beta1, double beta2, double eps, double lo, double hi, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FDWAVE_H */
