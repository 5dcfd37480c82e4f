/*
 * FP64 CPU oracle of the paper's own second-order flux-form scheme with variable
 * material (Herrmann, Buerchner, Kudela, Kollmannsberger, arXiv:2509.15744,
 * Sec. 3.1, Eqs. FDstencil1/FDstencil2), its exact discrete adjoint gradient and
 * the superposition approximation of Alg. 1 for both material fields.
 *
 * TEST INFRASTRUCTURE ONLY.  Like fdoracle.c this is the plain, slow reference
 * that the GPU library is checked against; only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Both equations of the paper have the form  m u_tt - div(b grad u) = f  with a
 * mass coefficient m and a stiffness coefficient b per cell:
 *   Eq. scalarwaveequation (rho-scaling):  m = gamma rho0,  b = gamma rho0 c0^2
 *   Eq. wavetopopt:                        m = 1/kappa,     b = 1/rho
 * Discretisation (Eqs. FDstencil1/2 in d dimensions, cell-centred grid):
 *
 *   u^{n+1}_i = 2 u^n_i - u^{n-1}_i + (dt^2 / m_i) ((L_b u^n)_i + f^n_i)
 *   (L_b u)_i = dx^-2 sum over the 2d neighbours j of i:  h(b_i, b_j) (u_j - u_i)
 *   h(p, q)   = 2 p q / (p + q)          (harmonic mean at the face, Sec. 3.1)
 *
 * Walls (Eq. BC, ghost cells whose material equals the boundary cell's, Sec. 3.1):
 * the ghost value mirrors the boundary cell, so a wall face carries no flux.
 * Time axis, point forces (f^n = wavelet[n] / dx^d), misfit and adjoint force are
 * those of fdoracle.c.
 *
 * Exact discrete gradient (Lagrangian of the scheme; the adjoint mu obeys the same
 * recursion backward with the force fdag = -(u - obs)/dt at the receivers,
 * mu^{nt} = 0, mu^{nt-1} = (dt^2/m) fdag^{nt}):
 *   dJ/dm_i   = -sum_{n=0}^{nt-1} (mu^{n+1} - mu^n)_i (u^{n+1} - u^n)_i
 *   dJ/dh_f   = (dt^2/dx^2) sum_{n=0}^{nt-1} (mu^n_j - mu^n_i)(u^n_j - u^n_i)   (face f = {i, j})
 *   dJ/db_i   = sum over the faces f of i:  dJ/dh_f * dh(b_i, b_j)/db_i,
 *               dh(p, q)/dp = 2 q^2 / (p + q)^2
 * These are the two terms of the paper's kernel (Eqs. kernel1, kernel2: the
 * time-derivative term for the mass coefficient, the gradient term for the
 * stiffness coefficient) in discrete form.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;
    long n[3];
    long stride[3];
    long ncell;
    double dx;
} vgrid_t;

static int make_vgrid(vgrid_t* g, int ndim, const long* shape, double dx)
{
    if (ndim < 1 || ndim > 3 || !(dx > 0.0)) return -1;
    g->ndim = ndim;
    for (int ax = 0; ax < 3; ++ax) g->n[ax] = ax < ndim ? shape[ax] : 1;
    for (int ax = 0; ax < ndim; ++ax)
        if (g->n[ax] < 1) return -1;
    g->stride[2] = 1;
    g->stride[1] = g->n[2];
    g->stride[0] = g->n[1] * g->n[2];
    g->ncell = g->n[0] * g->n[1] * g->n[2];
    g->dx = dx;
    return 0;
}

static double hmean(double p, double q) { return 2.0 * p * q / (p + q); }

/* Neighbour of `cell` one step along `ax` in direction `dir` (+1 or -1), or -1 at a
 * wall (the ghost there mirrors the cell itself). */
static long neighbour(const vgrid_t* g, long cell, int ax, int dir)
{
    const long coord = (cell / g->stride[ax]) % g->n[ax];
    const long c2 = coord + dir;
    if (c2 < 0 || c2 >= g->n[ax]) return -1;
    return cell + dir * g->stride[ax];
}

/* (L_b u) at one cell. */
static double vlap_at(const vgrid_t* g, const double* b, const double* u, long i)
{
    double s = 0.0;
    for (int ax = 0; ax < g->ndim; ++ax)
        for (int dir = -1; dir <= 1; dir += 2) {
            const long j = neighbour(g, i, ax, dir);
            if (j < 0) continue;   /* ghost = mirror of u_i: zero flux */
            s += hmean(b[i], b[j]) * (u[j] - u[i]);
        }
    return s / (g->dx * g->dx);
}

void orc_vd_operator(int ndim, const long* shape, double dx, const double* b, const double* u,
                     double* out)
{
    vgrid_t g;
    if (make_vgrid(&g, ndim, shape, dx)) return;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g.ncell; ++i) out[i] = vlap_at(&g, b, u, i);
}

/* One step: next = 2 cur - prev + (dt^2/m) L_b cur (point forces added after). */
static void vstep(const vgrid_t* g, const double* m, const double* b, double dt,
                  const double* prev, const double* cur, double* next)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g->ncell; ++i)
        next[i] = 2.0 * cur[i] - prev[i] + dt * dt / m[i] * vlap_at(g, b, cur, i);
}

static void vforces(const double* m, double dt, double* next, int npt, const long* cell,
                    const double* val, double scale)
{
    for (int q = 0; q < npt; ++q) next[cell[q]] += dt * dt / m[cell[q]] * (val[q] * scale);
}

static double vinv_volume(const vgrid_t* g)
{
    double v = 1.0;
    for (int ax = 0; ax < g->ndim; ++ax) v *= g->dx;
    return 1.0 / v;
}

/* sum over the faces of cell i of dh/db_i * (a_j - a_i)(c_j - c_i) for two fields a, c. */
static double face_term(const vgrid_t* g, const double* b, const double* a, const double* c, long i);

/* The two kernel terms of one field with itself (Eqs. kernel1/kernel2 in discrete
 * form): Km gains the mass term of the interval (a^{n+1}, a^n), sum of squared level
 * differences; Kb gains the stiffness term of level a^n, sum over the faces of dh/db
 * times the squared face difference.  Either level may be NULL (that term is skipped). */
static void vkernel_terms(const vgrid_t* g, const double* b, const double* a_next, const double* a_cur,
                          const double* a_level, double* Km, double* Kb)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g->ncell; ++i) {
        if (a_next) Km[i] += (a_next[i] - a_cur[i]) * (a_next[i] - a_cur[i]);
        if (a_level) Kb[i] += face_term(g, b, a_level, a_level, i);
    }
}

/* The forward problem forward in time from two zero levels.  traces [nt][nrec], hist
 * [(nt+1)][ncell] (levels 0..nt), last2 [2][ncell] (u^{nt-1}, u^nt) may be NULL; with
 * Km and Kb (both or neither) the kernel terms of u with itself are added: the mass
 * term over the nt intervals [n, n+1], the stiffness term over the levels 1..nt-1
 * (level 0 is zero; level nt is shared with the superposed field, whose end level it
 * is, so it cancels in their difference). */
static int vd_forward_solve(const vgrid_t* g, const double* m, const double* b, double dt, int nt,
                            int nsrc, const long* src, const double* wavelet, int nrec, const long* rec,
                            double* traces, double* hist, double* last2, double* Km, double* Kb)
{
    double* um = calloc(g->ncell, sizeof(double));
    double* u0 = calloc(g->ncell, sizeof(double));
    double* up = calloc(g->ncell, sizeof(double));
    if (!um || !u0 || !up) { free(um); free(u0); free(up); return -2; }
    const double vol = vinv_volume(g);
    if (hist) memset(hist, 0, sizeof(double) * g->ncell);
    for (int n = 0; n < nt; ++n) {
        vstep(g, m, b, dt, um, u0, up);
        vforces(m, dt, up, nsrc, src, wavelet + (long)n * nsrc, vol);
        if (traces)
            for (int q = 0; q < nrec; ++q) traces[(long)n * nrec + q] = up[rec[q]];
        if (hist) memcpy(hist + (long)(n + 1) * g->ncell, up, sizeof(double) * g->ncell);
        if (Km) vkernel_terms(g, b, up, u0, n >= 1 ? u0 : NULL, Km, Kb);
        double* t = um; um = u0; u0 = up; up = t;
    }
    if (last2) {
        memcpy(last2, um, sizeof(double) * g->ncell);
        memcpy(last2 + g->ncell, u0, sizeof(double) * g->ncell);
    }
    free(um); free(u0); free(up);
    return 0;
}

/* Forward solve: traces [nt][nrec] (may be NULL), hist [(nt+1)][ncell] levels 0..nt
 * (may be NULL), last2 [2][ncell] u^{nt-1}, u^nt (may be NULL). */
int orc_vd_forward(int ndim, const long* shape, double dx, const double* m, const double* b,
                   double dt, int nt, int nsrc, const long* src, const double* wavelet,
                   int nrec, const long* rec, double* traces, double* hist, double* last2)
{
    vgrid_t g;
    if (make_vgrid(&g, ndim, shape, dx) || nt < 1) return -1;
    return vd_forward_solve(&g, m, b, dt, nt, nsrc, src, wavelet, nrec, rec, traces, hist, last2, NULL, NULL);
}

/* Adjoint sweep: mu^{nt} = mu^{nt+1} = 0, mu^{j-1} = 2 mu^j - mu^{j+1} +
 * (dt^2/m)(L_b mu^j + fdag^j), j = nt..1, fdag [nt][nrec] injected at the receivers
 * without 1/dx^d.  hist [(nt+1)][ncell] receives mu^0..mu^nt (may be NULL). */
int orc_vd_adjoint(int ndim, const long* shape, double dx, const double* m, const double* b,
                   double dt, int nt, int nrec, const long* rec, const double* fdag, double* hist)
{
    vgrid_t g;
    if (make_vgrid(&g, ndim, shape, dx) || nt < 1) return -1;
    double* mp = calloc(g.ncell, sizeof(double));
    double* m0 = calloc(g.ncell, sizeof(double));
    double* mm = calloc(g.ncell, sizeof(double));
    if (!mp || !m0 || !mm) { free(mp); free(m0); free(mm); return -2; }
    if (hist) memset(hist + (long)nt * g.ncell, 0, sizeof(double) * g.ncell);
    for (int j = nt; j >= 1; --j) {
        vstep(&g, m, b, dt, mp, m0, mm);
        vforces(m, dt, mm, nrec, rec, fdag + (long)(j - 1) * nrec, 1.0);
        if (hist) memcpy(hist + (long)(j - 1) * g.ncell, mm, sizeof(double) * g.ncell);
        double* t = mp; mp = m0; m0 = mm; mm = t;
    }
    free(mp); free(m0); free(mm);
    return 0;
}

/* sum over the faces of cell i of dh/db_i * (a_j - a_i)(c_j - c_i) for two fields a, c. */
static double face_term(const vgrid_t* g, const double* b, const double* a, const double* c, long i)
{
    double s = 0.0;
    for (int ax = 0; ax < g->ndim; ++ax)
        for (int dir = -1; dir <= 1; dir += 2) {
            const long j = neighbour(g, i, ax, dir);
            if (j < 0) continue;
            const double w = 2.0 * b[j] * b[j] / ((b[i] + b[j]) * (b[i] + b[j]));
            s += w * (a[j] - a[i]) * (c[j] - c[i]);
        }
    return s;
}

/* Exact discrete gradient with stored history: grad_m, grad_b [ncell] (formulas in
 * the header).  s2_m, s2_b (may be NULL) receive the k^2 terms of the superposition,
 * sum_n (mu^{n+1} - mu^n)^2 and sum_{n>=1} sum_faces dh/db (mu_j^n - mu_i^n)^2. */
int orc_vd_exact_gradient(int ndim, const long* shape, double dx, const double* m, const double* b,
                          double dt, int nt, int nsrc, const long* src, const double* wavelet,
                          int nrec, const long* rec, const double* obs, double* grad_m,
                          double* grad_b, double* J, double* s2_m, double* s2_b, double* traces_out)
{
    vgrid_t g;
    if (make_vgrid(&g, ndim, shape, dx) || nt < 1) return -1;
    const long N = g.ncell;
    double* uh = malloc(sizeof(double) * (size_t)(nt + 1) * N);
    double* mh = malloc(sizeof(double) * (size_t)(nt + 1) * N);
    double* tr = malloc(sizeof(double) * (size_t)nt * (nrec > 0 ? nrec : 1));
    double* fd = malloc(sizeof(double) * (size_t)nt * (nrec > 0 ? nrec : 1));
    if (!uh || !mh || !tr || !fd) { free(uh); free(mh); free(tr); free(fd); return -2; }
    int rc = orc_vd_forward(ndim, shape, dx, m, b, dt, nt, nsrc, src, wavelet, nrec, rec, tr, uh, NULL);
    if (!rc) {
        double s = 0.0;
        for (long q = 0; q < (long)nt * nrec; ++q) {
            const double rho = tr[q] - obs[q];
            s += rho * rho;
            fd[q] = -rho / dt;
        }
        if (J) *J = 0.5 * dt * s;
        rc = orc_vd_adjoint(ndim, shape, dx, m, b, dt, nt, nrec, rec, fd, mh);
    }
    if (!rc) {
        const double fac = dt * dt / (dx * dx);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            double gm = 0.0, gb = 0.0, sm = 0.0, sb = 0.0;
            for (int n = 0; n < nt; ++n) {
                const double* u0 = uh + (long)n * N;
                const double* u1 = uh + (long)(n + 1) * N;
                const double* m0 = mh + (long)n * N;
                const double* m1 = mh + (long)(n + 1) * N;
                gm -= (m1[i] - m0[i]) * (u1[i] - u0[i]);
                sm += (m1[i] - m0[i]) * (m1[i] - m0[i]);
                gb += face_term(&g, b, m0, u0, i);
                if (n >= 1) sb += face_term(&g, b, m0, m0, i);
            }
            grad_m[i] = gm;
            grad_b[i] = fac * gb;
            if (s2_m) s2_m[i] = sm;
            if (s2_b) s2_b[i] = sb;
        }
        if (traces_out) memcpy(traces_out, tr, sizeof(double) * (size_t)nt * nrec);
    }
    free(uh); free(mh); free(tr); free(fd);
    return rc;
}

/* The superposed field v = u + k mu solved backward in time (Sec. 4, Eqs.
 * superposedPDE2/superposedforce: the forward operator with the force f + k fdag) from
 * its end levels v^nt (v_hi) and v^{nt-1} (v_lo), both overwritten:
 *   v^{j-1} = 2 v^j - v^{j+1} + (dt^2/m)(L_b v^j + f^j + k fdag^j),  j = nt-1..1,
 * f^j = wavelet row j over the cell volume, fdag^j = row j-1 of fdag at the receivers.
 * Km, Kb gain the kernel terms of v with itself over the same intervals (all nt) and
 * levels (1..nt-1) as the forward field's. */
static int vd_superposed_solve(const vgrid_t* g, const double* m, const double* b, double dt, int nt,
                               int nsrc, const long* src, const double* wavelet, int nrec, const long* rec,
                               const double* fdag, double k, double* v_hi, double* v_lo, double* Km,
                               double* Kb)
{
    double* buf = malloc(sizeof(double) * g->ncell);
    if (!buf) return -2;
    const double vol = vinv_volume(g);
    double* vp = v_hi;   /* v^{j+1} */
    double* v0 = v_lo;   /* v^j */
    double* vm = buf;    /* v^{j-1} */
    vkernel_terms(g, b, vp, v0, NULL, Km, Kb);   /* interval [nt-1, nt] */
    for (int j = nt - 1; j >= 1; --j) {
        vstep(g, m, b, dt, vp, v0, vm);
        vforces(m, dt, vm, nsrc, src, wavelet + (long)j * nsrc, vol);
        vforces(m, dt, vm, nrec, rec, fdag + (long)(j - 1) * nrec, k);
        vkernel_terms(g, b, v0, vm, v0, Km, Kb);   /* interval [j-1, j], level j */
        double* t = vp; vp = v0; v0 = vm; vm = t;
    }
    free(buf);
    return 0;
}

/* The memory-efficient sensitivity of Sec. 4 (Alg. 1) for both material fields,
 * from its equations: the forward problem with the kernel terms of u with itself,
 * the cost (Eq. cost1) and adjoint force fdag = -(u - obs)/dt (Eq. adjointSource1),
 * the superposed field v = u + k mu backward from v^nt = u^nt, v^{nt-1} = u^{nt-1} +
 * k (dt^2/m) fdag^nt (the discrete adjoint's end levels are mu^nt = 0, mu^{nt-1} =
 * (dt^2/m) fdag^nt) with the kernel terms of v with itself, and the mixed kernel of Eq.
 * superposedkernel per term.  With the mass term written as a sum of squares
 * (Km = -K, so its difference changes sign) and the stiffness term carrying the
 * scheme's dt^2/dx^2:
 *   dJ/dm ~ (Km(u,u) - Km(v,v)) / (2k),   dJ/db ~ -(dt^2/dx^2)(Kb(u,u) - Kb(v,v)) / (2k). */
int orc_vd_superposition(int ndim, const long* shape, double dx, const double* m, const double* b,
                         double dt, int nt, int nsrc, const long* src, const double* wavelet,
                         int nrec, const long* rec, const double* obs, double k, double* grad_m,
                         double* grad_b, double* J, double* traces_out)
{
    vgrid_t g;
    if (make_vgrid(&g, ndim, shape, dx) || nt < 1 || !(k != 0.0)) return -1;
    const long N = g.ncell;
    const size_t nq = (size_t)nt * (nrec > 0 ? nrec : 1);
    double* kmu = calloc(N, sizeof(double));
    double* kbu = calloc(N, sizeof(double));
    double* kmv = calloc(N, sizeof(double));
    double* kbv = calloc(N, sizeof(double));
    double* ends = malloc(sizeof(double) * 2 * N);   /* u^{nt-1}, u^nt */
    double* tr = malloc(sizeof(double) * nq);
    double* fd = malloc(sizeof(double) * nq);
    int rc = (!kmu || !kbu || !kmv || !kbv || !ends || !tr || !fd) ? -2 : 0;
    if (!rc) rc = vd_forward_solve(&g, m, b, dt, nt, nsrc, src, wavelet, nrec, rec, tr, NULL, ends, kmu, kbu);
    if (!rc) {
        double s = 0.0;
        for (long q = 0; q < (long)nt * nrec; ++q) {
            const double rho = tr[q] - obs[q];
            s += rho * rho;
            fd[q] = -rho / dt;
        }
        if (J) *J = 0.5 * dt * s;
        if (traces_out) memcpy(traces_out, tr, sizeof(double) * (size_t)nt * nrec);
        vforces(m, dt, ends, nrec, rec, fd + (long)(nt - 1) * nrec, k);   /* v^{nt-1} */
        rc = vd_superposed_solve(&g, m, b, dt, nt, nsrc, src, wavelet, nrec, rec, fd, k, ends + N, ends,
                                 kmv, kbv);
    }
    if (!rc) {
        const double fac = dt * dt / (dx * dx);
        for (long i = 0; i < N; ++i) {
            grad_m[i] = (kmu[i] - kmv[i]) / (2.0 * k);
            grad_b[i] = -fac * (kbu[i] - kbv[i]) / (2.0 * k);
        }
    }
    free(kmu); free(kbu); free(kmv); free(kbv); free(ends); free(tr); free(fd);
    return rc;
}
