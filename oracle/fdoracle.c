/*
 * FP64 CPU oracle for the memory-efficient superposition adjoint method
 * (Herrmann, Buerchner, Kudela, Kollmannsberger, arXiv:2509.15744).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Everything is double precision, with plain loops; OpenMP only distributes
 * independent cells over threads (no cell's arithmetic is reordered).
 *
 * Discretisation (paper Sec. 3.1, Eq. FDstencil2 with rho^-1 = 1 and
 * kappa = c^2, extended to a 2r-th order central Laplacian):
 *
 *   u^{n+1} = 2 u^n - u^{n-1} + coef * (L u^n + f^n),   coef = dt^2 c^2
 *
 *   (L u)_i = dx^-2 sum_axes sum_{j=1..r} a_j [(u_{i+j} - u_i) + (u_{i-j} - u_i)]
 *
 * Homogeneous Neumann walls (paper Eq. BC) through ghost cells (paper
 * Sec. 3.1): the grid is cell-centred and a ghost index mirrors about the
 * half-cell face, -1-j -> j and n+j -> n-1-j.
 *
 * Time origin: u^{-1} = u^0 = 0 (paper Eq. IC; Alg. 1 starts from two zero
 * levels).  Forward steps n = 0..nt-1 produce u^1..u^nt; the point force at
 * step n is f^n = sum_s wavelet[n][s] delta_{x_s} / dx^d (paper Eq. source1
 * with a discrete delta).  Receivers record u^1..u^nt; traces row n-1 holds
 * level n.
 *
 * Misfit (paper Eq. cost1, time integral as dt * sum):
 *   J = dt/2 sum_{n=1..nt} sum_r (u^n(x_r) - obs^n_r)^2
 * Adjoint force (paper Eq. adjointSource1, scaled so that it enters the same
 * step as f):  fdag^n_r = -(u^n(x_r) - obs^n_r) / dt, injected without 1/dx^d.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the oracle's parallel loops use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set that number (timing the oracle single-threaded); returns the previous one. */
int orc_set_threads(int n)
{
    const int prev = orc_num_threads();
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return prev;
}

typedef struct {
    int ndim;      /* 1, 2 or 3 */
    long n[3];     /* extents, axis 0 slowest; unused trailing axes have extent 1 */
    long stride[3];
    long ncell;
    double dx;
    int r;         /* stencil radius: order / 2 */
    double w[9];   /* w[j] = a_j / dx^2, j = 1..r */
} grid_t;

static int make_grid(grid_t* g, int ndim, const long* shape, double dx, int r, const double* a)
{
    if (ndim < 1 || ndim > 3 || r < 1 || r > 8 || !(dx > 0.0)) return -1;
    g->ndim = ndim;
    for (int ax = 0; ax < 3; ++ax) g->n[ax] = ax < ndim ? shape[ax] : 1;
    for (int ax = 0; ax < ndim; ++ax)
        if (g->n[ax] < r) return -1;   /* the single mirror needs n >= r */
    g->stride[2] = 1;
    g->stride[1] = g->n[2];
    g->stride[0] = g->n[1] * g->n[2];
    g->ncell = g->n[0] * g->n[1] * g->n[2];
    g->dx = dx;
    g->r = r;
    for (int j = 1; j <= r; ++j) g->w[j] = a[j - 1] / (dx * dx);
    return 0;
}

/* Ghost cell index: half-sample mirror about the wall faces. */
static long mirror(long i, long n)
{
    if (i < 0) return -1 - i;
    if (i >= n) return 2 * n - 1 - i;
    return i;
}

/* (L u) at one cell, straight from the definition above. */
static double lap_at(const grid_t* g, const double* u, long cell)
{
    long pos[3];
    long rem = cell;
    for (int ax = 0; ax < 3; ++ax) {
        pos[ax] = rem / g->stride[ax];
        rem -= pos[ax] * g->stride[ax];
    }
    const double ui = u[cell];
    double s = 0.0;
    for (int ax = 0; ax < g->ndim; ++ax) {
        for (int j = 1; j <= g->r; ++j) {
            long ip = mirror(pos[ax] + j, g->n[ax]);
            long im = mirror(pos[ax] - j, g->n[ax]);
            double up = u[cell + (ip - pos[ax]) * g->stride[ax]];
            double um = u[cell + (im - pos[ax]) * g->stride[ax]];
            s += g->w[j] * ((up - ui) + (um - ui));
        }
    }
    return s;
}

void orc_laplacian(int ndim, const long* shape, double dx, int r, const double* a,
                   const double* u, double* out)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a)) return;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g.ncell; ++i) out[i] = lap_at(&g, u, i);
}

/* propagateStep (paper Alg. 1): u_next = 2 u_cur - u_prev + coef * L u_cur.
 * Point forces are added afterwards by add_point_forces(). */
static void propagate_step(const grid_t* g, const double* coef, const double* u_prev,
                           const double* u_cur, double* u_next)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g->ncell; ++i)
        u_next[i] = 2.0 * u_cur[i] - u_prev[i] + coef[i] * lap_at(g, u_cur, i);
}

/* u_next += coef * (point force), one force value per listed cell. */
static void add_point_forces(const double* coef, double* u_next, int npt, const long* cell,
                             const double* value, double scale)
{
    for (int p = 0; p < npt; ++p) u_next[cell[p]] += coef[cell[p]] * value[p] * scale;
}

static double inv_cell_volume(const grid_t* g)
{
    return 1.0 / pow(g->dx, (double)g->ndim);
}

/* Source-free propagation from given levels; on return u_prev holds level
 * nsteps-1 and u_cur level nsteps (relative to the inputs as levels -1, 0). */
int orc_propagate(int ndim, const long* shape, double dx, int r, const double* a,
                  const double* coef, double* u_prev, double* u_cur, int nsteps)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a)) return -1;
    double* u_next = malloc(sizeof(double) * g.ncell);
    if (!u_next) return -2;
    for (int n = 0; n < nsteps; ++n) {
        propagate_step(&g, coef, u_prev, u_cur, u_next);
        memcpy(u_prev, u_cur, sizeof(double) * g.ncell);
        memcpy(u_cur, u_next, sizeof(double) * g.ncell);
    }
    free(u_next);
    return 0;
}

static double* coef_from_speed(const grid_t* g, const double* c, double dt)
{
    double* coef = malloc(sizeof(double) * g->ncell);
    if (!coef) return NULL;
    for (long i = 0; i < g->ncell; ++i) coef[i] = dt * dt * c[i] * c[i];
    return coef;
}

/* Mass-term kernel of one time interval (Eq. kernel2 in the parameter m = 1/c^2, its
 * time derivatives as differences of consecutive levels): for a level pair
 * (a^{n+1}, a^n) of one field, K(a,a)_i gains -(a^{n+1} - a^n)_i^2. */
static void kernel_interval(long N, const double* a_next, const double* a_cur, double* K)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        const double d = a_next[i] - a_cur[i];
        K[i] -= d * d;
    }
}

/* The forward problem solved forward in time from two zero levels.  traces
 * [nt][nrec], hist [(nt+1)][ncell] (levels 0..nt), last2 [2][ncell] (u^{nt-1}, u^nt)
 * and Kuu [ncell] (K(u,u) over the nt intervals [n, n+1], added to what it holds)
 * may each be NULL. */
static int forward_solve(const grid_t* g, const double* coef, int nt, int nsrc, const long* src,
                         const double* wavelet, int nrec, const long* rec, double* traces,
                         double* hist, double* last2, double* Kuu)
{
    double* um = calloc(g->ncell, sizeof(double));   /* u^{n-1} */
    double* u0 = calloc(g->ncell, sizeof(double));   /* u^n     */
    double* up = calloc(g->ncell, sizeof(double));   /* u^{n+1} */
    if (!um || !u0 || !up) { free(um); free(u0); free(up); return -2; }
    const double vol = inv_cell_volume(g);
    if (hist) memset(hist, 0, sizeof(double) * g->ncell);   /* level 0 */
    for (int n = 0; n < nt; ++n) {
        propagate_step(g, coef, um, u0, up);
        add_point_forces(coef, up, nsrc, src, wavelet + (long)n * nsrc, vol);
        if (traces)
            for (int q = 0; q < nrec; ++q) traces[(long)n * nrec + q] = up[rec[q]];
        if (hist) memcpy(hist + (long)(n + 1) * g->ncell, up, sizeof(double) * g->ncell);
        if (Kuu) kernel_interval(g->ncell, up, u0, Kuu);
        double* t = um; um = u0; u0 = up; up = t;
    }
    if (last2) {
        memcpy(last2, um, sizeof(double) * g->ncell);
        memcpy(last2 + g->ncell, u0, sizeof(double) * g->ncell);
    }
    free(um); free(u0); free(up);
    return 0;
}

/* Forward solve.  traces [nt][nrec] (may be NULL); hist [(nt+1)][ncell] holds
 * levels 0..nt (may be NULL); last2 [2][ncell] receives u^{nt-1}, u^nt (may be
 * NULL). */
int orc_forward(int ndim, const long* shape, double dx, int r, const double* a,
                const double* c, double dt, int nt,
                int nsrc, const long* src, const double* wavelet,
                int nrec, const long* rec,
                double* traces, double* hist, double* last2)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a) || nt < 1) return -1;
    double* coef = coef_from_speed(&g, c, dt);
    if (!coef) return -2;
    const int rc = forward_solve(&g, coef, nt, nsrc, src, wavelet, nrec, rec, traces, hist, last2, NULL);
    free(coef);
    return rc;
}

/* J = dt/2 sum (traces - obs)^2 in index order; resid (may be NULL) = traces - obs. */
double orc_misfit(int nt, int nrec, double dt, const double* traces, const double* obs,
                  double* resid)
{
    double s = 0.0;
    for (long i = 0; i < (long)nt * nrec; ++i) {
        double rho = traces[i] - obs[i];
        if (resid) resid[i] = rho;
        s += rho * rho;
    }
    return 0.5 * dt * s;
}

/* Backward (adjoint) sweep of the same operator (the problem is self-adjoint,
 * paper Sec. 2.2, Eq. adjointequation1):
 *   mu^{nt} = mu^{nt+1} = 0,
 *   mu^{j-1} = 2 mu^j - mu^{j+1} + coef * (L mu^j + fdag^j),  j = nt..1,
 * with fdag [nt][nrec] (row j-1 = force at level j) injected at the receivers
 * without cell-volume scaling.  hist [(nt+1)][ncell] receives mu^0..mu^nt (may
 * be NULL); mu_src [nt][nsrc] receives mu^n at the source cells for n = 0..nt-1
 * (may be NULL). */
int orc_adjoint(int ndim, const long* shape, double dx, int r, const double* a,
                const double* c, double dt, int nt,
                int nrec, const long* rec, const double* fdag,
                double* hist, int nsrc, const long* src, double* mu_src)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a) || nt < 1) return -1;
    double* coef = coef_from_speed(&g, c, dt);
    double* mp = calloc(g.ncell, sizeof(double));   /* mu^{j+1} */
    double* m0 = calloc(g.ncell, sizeof(double));   /* mu^j     */
    double* mm = calloc(g.ncell, sizeof(double));   /* mu^{j-1} */
    if (!coef || !mp || !m0 || !mm) { free(coef); free(mp); free(m0); free(mm); return -2; }
    if (hist) memset(hist + (long)nt * g.ncell, 0, sizeof(double) * g.ncell);
    for (int j = nt; j >= 1; --j) {
        propagate_step(&g, coef, mp, m0, mm);
        add_point_forces(coef, mm, nrec, rec, fdag + (long)(j - 1) * nrec, 1.0);
        if (hist) memcpy(hist + (long)(j - 1) * g.ncell, mm, sizeof(double) * g.ncell);
        if (mu_src)
            for (int s = 0; s < nsrc; ++s) mu_src[(long)(j - 1) * nsrc + s] = mm[src[s]];
        double* t = mp; mp = m0; m0 = mm; mm = t;
    }
    free(coef); free(mp); free(m0); free(mm);
    return 0;
}

/* Exact discrete adjoint gradient with the full forward history stored.
 *   dJ/dm_i = -sum_{n=0}^{nt-1} (mu^{n+1} - mu^n)_i (u^{n+1} - u^n)_i,  m = 1/c^2
 *   dJ/dc_i = -(2 / c_i^3) dJ/dm_i
 * (paper Eq. kernel2, mass term, as the discrete bilinear form in the time
 * differences; Eq. gradientgamma per grid point).  sum_dmu2 (may be NULL)
 * receives sum_n (mu^{n+1} - mu^n)_i^2, the k^2 term of Eq. superposedkernel1. */
int orc_exact_gradient(int ndim, const long* shape, double dx, int r, const double* a,
                       const double* c, double dt, int nt,
                       int nsrc, const long* src, const double* wavelet,
                       int nrec, const long* rec, const double* obs,
                       double* grad_c, double* J, double* sum_dmu2, double* traces_out)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a) || nt < 1) return -1;
    const long N = g.ncell;
    double* uh = malloc(sizeof(double) * (size_t)(nt + 1) * N);
    double* mh = malloc(sizeof(double) * (size_t)(nt + 1) * N);
    double* tr = malloc(sizeof(double) * (size_t)nt * nrec);
    double* fd = malloc(sizeof(double) * (size_t)nt * nrec);
    if (!uh || !mh || !tr || !fd) { free(uh); free(mh); free(tr); free(fd); return -2; }
    int rc = orc_forward(ndim, shape, dx, r, a, c, dt, nt, nsrc, src, wavelet, nrec, rec,
                         tr, uh, NULL);
    if (!rc) {
        double Jv = orc_misfit(nt, nrec, dt, tr, obs, fd);
        if (J) *J = Jv;
        for (long i = 0; i < (long)nt * nrec; ++i) fd[i] = -fd[i] / dt;
        rc = orc_adjoint(ndim, shape, dx, r, a, c, dt, nt, nrec, rec, fd, mh, 0, NULL, NULL);
    }
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            double gm = 0.0, s2 = 0.0;
            for (int n = 0; n < nt; ++n) {
                double du = uh[(long)(n + 1) * N + i] - uh[(long)n * N + i];
                double dm = mh[(long)(n + 1) * N + i] - mh[(long)n * N + i];
                gm -= dm * du;
                s2 += dm * dm;
            }
            grad_c[i] = -2.0 / (c[i] * c[i] * c[i]) * gm;
            if (sum_dmu2) sum_dmu2[i] = s2;
        }
        if (traces_out) memcpy(traces_out, tr, sizeof(double) * (size_t)nt * nrec);
    }
    free(uh); free(mh); free(tr); free(fd);
    return rc;
}

/* The exact discrete adjoint gradient of orc_exact_gradient with the forward
 * history replaced by checkpoints: the pair (u^{a-1}, u^a) is kept every `seg`
 * levels, and each segment of levels a..b is recomputed from its checkpoint
 * just before the backward sweep crosses it (uniform checkpointing, one extra
 * forward solve).  Same outputs; memory ~ (2 nt/seg + seg) grids. */
int orc_exact_gradient_ckpt(int ndim, const long* shape, double dx, int r, const double* a,
                            const double* c, double dt, int nt,
                            int nsrc, const long* src, const double* wavelet,
                            int nrec, const long* rec, const double* obs, int seg,
                            double* grad_c, double* J, double* sum_dmu2, double* traces_out)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a) || nt < 1 || seg < 1) return -1;
    const long N = g.ncell;
    const double vol = inv_cell_volume(&g);
    const int nck = (nt + seg - 1) / seg;          /* checkpoints at a = 0, seg, 2 seg, ... */
    double* coef = coef_from_speed(&g, c, dt);
    double* ck = malloc(sizeof(double) * (size_t)nck * 2 * N);
    double* sg = malloc(sizeof(double) * (size_t)(seg + 1) * N);   /* levels a..b */
    double* um = calloc(N, sizeof(double));
    double* u0 = calloc(N, sizeof(double));
    double* up = calloc(N, sizeof(double));
    double* fdag = malloc(sizeof(double) * (size_t)nt * nrec);
    double* tr = malloc(sizeof(double) * (size_t)nt * nrec);
    double* gm = calloc(N, sizeof(double));
    double* s2 = calloc(N, sizeof(double));
    if (!coef || !ck || !sg || !um || !u0 || !up || !fdag || !tr || !gm || !s2) {
        free(coef); free(ck); free(sg); free(um); free(u0); free(up); free(fdag); free(tr);
        free(gm); free(s2);
        return -2;
    }
    /* forward solve, keeping checkpoints and the traces */
    for (int n = 0; n < nt; ++n) {
        if (n % seg == 0) {
            memcpy(ck + (size_t)(n / seg) * 2 * N, um, sizeof(double) * N);
            memcpy(ck + (size_t)(n / seg) * 2 * N + N, u0, sizeof(double) * N);
        }
        propagate_step(&g, coef, um, u0, up);
        add_point_forces(coef, up, nsrc, src, wavelet + (long)n * nsrc, vol);
        for (int q = 0; q < nrec; ++q) tr[(long)n * nrec + q] = up[rec[q]];
        double* t = um; um = u0; u0 = up; up = t;
    }
    double Jv = orc_misfit(nt, nrec, dt, tr, obs, fdag);
    for (long i = 0; i < (long)nt * nrec; ++i) fdag[i] = -fdag[i] / dt;

    /* backward sweep segment by segment: mu^{j-1} from mu^j, mu^{j+1} */
    double* mp = um; double* m0 = u0; double* mm = up;   /* reuse the three grids */
    memset(mp, 0, sizeof(double) * N);
    memset(m0, 0, sizeof(double) * N);
    for (int s = nck - 1; s >= 0; --s) {
        const int lo = s * seg;
        const int hi = lo + seg < nt ? lo + seg : nt;
        /* recompute levels lo..hi from the checkpoint (u^{lo-1}, u^lo) */
        double* wm = malloc(sizeof(double) * N);
        if (!wm) { Jv = NAN; break; }
        memcpy(wm, ck + (size_t)s * 2 * N, sizeof(double) * N);
        memcpy(sg, ck + (size_t)s * 2 * N + N, sizeof(double) * N);
        for (int n = lo; n < hi; ++n) {
            double* cur = sg + (size_t)(n - lo) * N;
            double* nxt = sg + (size_t)(n - lo + 1) * N;
            const double* prv = n == lo ? wm : sg + (size_t)(n - lo - 1) * N;
            propagate_step(&g, coef, prv, cur, nxt);
            add_point_forces(coef, nxt, nsrc, src, wavelet + (long)n * nsrc, vol);
        }
        free(wm);
        for (int j = hi; j > lo; --j) {
            propagate_step(&g, coef, mp, m0, mm);
            add_point_forces(coef, mm, nrec, rec, fdag + (long)(j - 1) * nrec, 1.0);
            const double* uj = sg + (size_t)(j - lo) * N;
            const double* uj1 = sg + (size_t)(j - 1 - lo) * N;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < N; ++i) {
                double du = uj[i] - uj1[i];
                double dm = m0[i] - mm[i];    /* mu^j - mu^{j-1} */
                gm[i] -= dm * du;
                s2[i] += dm * dm;
            }
            double* t = mp; mp = m0; m0 = mm; mm = t;
        }
    }
    for (long i = 0; i < N; ++i) {
        grad_c[i] = -2.0 / (c[i] * c[i] * c[i]) * gm[i];
        if (sum_dmu2) sum_dmu2[i] = s2[i];
    }
    if (J) *J = Jv;
    if (traces_out) memcpy(traces_out, tr, sizeof(double) * (size_t)nt * nrec);
    free(coef); free(ck); free(sg); free(um); free(u0); free(up); free(fdag); free(tr);
    free(gm); free(s2);
    return isnan(Jv) ? -2 : 0;
}

/* The superposed problem solved backward in time (Sec. 4, Eq. superposedPDE: the
 * same operator as the forward problem, driven by the superposed force of Eq.
 * superposedforce, f^s = f + k fdag, with fdag of Eq. adjointSource1):
 *   v^{j-1} = 2 v^j - v^{j+1} + coef (L v^j + f^j + k fdag^j),  j = nt-1..1,
 * from the end levels v^nt (v_hi) and v^{nt-1} (v_lo), which the call overwrites.
 * f^j is the source term of level j (wavelet row j over the cell volume), fdag^j the
 * adjoint force of level j (row j-1 of fdag [nt][nrec], injected without a volume
 * factor).  Kvv [ncell] gains K(v,v) over all nt intervals [j-1, j], j = nt..1. */
static int superposed_solve(const grid_t* g, const double* coef, int nt, int nsrc, const long* src,
                            const double* wavelet, int nrec, const long* rec, const double* fdag,
                            double k, double* v_hi, double* v_lo, double* Kvv)
{
    double* buf = malloc(sizeof(double) * g->ncell);
    if (!buf) return -2;
    const double vol = inv_cell_volume(g);
    double* vp = v_hi;   /* v^{j+1} */
    double* v0 = v_lo;   /* v^j     */
    double* vm = buf;    /* v^{j-1} */
    kernel_interval(g->ncell, vp, v0, Kvv);   /* [nt-1, nt] */
    for (int j = nt - 1; j >= 1; --j) {
        propagate_step(g, coef, vp, v0, vm);
        add_point_forces(coef, vm, nsrc, src, wavelet + (long)j * nsrc, vol);
        add_point_forces(coef, vm, nrec, rec, fdag + (long)(j - 1) * nrec, k);
        kernel_interval(g->ncell, v0, vm, Kvv);   /* [j-1, j] */
        double* t = vp; vp = v0; v0 = vm; vm = t;
    }
    free(buf);
    return 0;
}

/* The memory-efficient sensitivity of Sec. 4 (Alg. 1) at factor k, assembled from
 * its equations:
 *   1. the forward problem with K(u,u), the kernel of the forward field with itself
 *      (it needs no stored history: each interval is added as the solve passes it);
 *   2. the cost (Eq. cost1) and the adjoint force fdag^n = -(u^n(x_r) - obs^n_r)/dt
 *      (Eq. adjointSource1);
 *   3. the superposed field v = u + k mu (mu the adjoint field), which obeys the
 *      forward operator with the force f + k fdag (Eqs. superposedPDE,
 *      superposedforce) and is solved backward in time from its end levels with
 *      K(v,v) accumulated on the way;
 *   4. the mixed kernel of Eq. superposedkernel, K~ = (K(v,v) - K(u,u)) / (2k), which
 *      approximates K(u,mu) = dJ/dm (Eq. superposedkernel1 without its k^2 term),
 *      and dJ/dc = -(2/c^3) dJ/dm (m = 1/c^2).
 * Kernel of a level sequence a with itself: K(a,a)_i = -sum_{n=0}^{nt-1} (a^{n+1} -
 * a^n)_i^2 (Eq. kernel2, mass term), over the same nt intervals for u and v.
 *
 * End levels of v: the adjoint field's end conditions are homogeneous (Eq.
 * ICadjoint), so the superposed end state is the forward one (Sec. 4); discretely the
 * adjoint recursion started from mu^{nt+1} = mu^nt = 0 has mu^{nt-1} = coef fdag^nt at
 * the receivers, so v^nt = u^nt and v^{nt-1} = u^{nt-1} + k coef fdag^nt, which keeps
 * v = u + k mu level by level.  traces [nt][nrec] may be NULL. */
int orc_superposition(int ndim, const long* shape, double dx, int r, const double* a,
                      const double* c, double dt, int nt,
                      int nsrc, const long* src, const double* wavelet,
                      int nrec, const long* rec, const double* obs, double k,
                      double* grad_c, double* J, double* traces)
{
    grid_t g;
    if (make_grid(&g, ndim, shape, dx, r, a) || nt < 1 || k == 0.0) return -1;
    const long N = g.ncell;
    double* coef = coef_from_speed(&g, c, dt);
    double* Kuu = calloc(N, sizeof(double));
    double* Kvv = calloc(N, sizeof(double));
    double* ends = malloc(sizeof(double) * 2 * N);                 /* u^{nt-1}, u^nt */
    double* tr = malloc(sizeof(double) * ((size_t)nt * nrec + 1));
    double* fdag = malloc(sizeof(double) * ((size_t)nt * nrec + 1)); /* row n-1: level n */
    int rc = (!coef || !Kuu || !Kvv || !ends || !tr || !fdag) ? -2 : 0;

    /* 1. forward problem and K(u,u) */
    if (!rc) rc = forward_solve(&g, coef, nt, nsrc, src, wavelet, nrec, rec, tr, NULL, ends, Kuu);
    if (!rc) {
        /* 2. cost and adjoint force */
        const double cost = orc_misfit(nt, nrec, dt, tr, obs, fdag);
        for (long q = 0; q < (long)nt * nrec; ++q) fdag[q] = -fdag[q] / dt;
        if (J) *J = cost;
        if (traces) memcpy(traces, tr, sizeof(double) * (size_t)nt * nrec);
        /* 3. superposed field from v^{nt-1} = u^{nt-1} + k coef fdag^nt, v^nt = u^nt */
        add_point_forces(coef, ends, nrec, rec, fdag + (long)(nt - 1) * nrec, k);
        rc = superposed_solve(&g, coef, nt, nsrc, src, wavelet, nrec, rec, fdag, k, ends + N, ends, Kvv);
    }
    if (!rc) {
        /* 4. mixed kernel and the gradient in c */
        for (long i = 0; i < N; ++i) {
            const double dJdm = (Kvv[i] - Kuu[i]) / (2.0 * k);
            grad_c[i] = -2.0 / (c[i] * c[i] * c[i]) * dJdm;
        }
    }
    free(coef); free(Kuu); free(Kvv); free(ends); free(tr); free(fdag);
    return rc;
}
