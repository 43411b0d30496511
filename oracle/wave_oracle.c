/*
 * Plain CPU oracle for the damped acoustic leapfrog scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper: "Seismic Inversion Example"):
 *   m u_tt + eta u_t - lap(u) = q           (equation "eqn:acoustic")
 * discretised as in the forward listing ("lst:wave"): central second
 * difference in time (u.dt2), a central first difference for u.dt (the
 * listing uses time_order=2; the stencil of u.dt is not printed, the central
 * one is the reading taken), order-2k central second differences in space
 * (u.laplace = sum of f.dx2 over the axes, Section "High-level API"), solved
 * for u.forward:
 *   u+ = (2 m u - (m - eta dt/2) u- + dt^2 L u) / (m + eta dt/2)
 * The adjoint ("lst:adjoint") flips the sign of the eta term and is solved
 * for v.backward, which gives the same update run backwards in time.
 * Sparse points (Section "Sparse point interpolation") are multilinear: a
 * point spreads into / samples from the 2^d nodes of its enclosing cell.
 *
 * Precision: every quantity is `real`, double by default; building with
 * -DORACLE_REAL_FLOAT gives the same loops in float, used only to measure the
 * FP32 round-off floor.  The interface is always double.
 *
 * Deliberately plain: triple loops, bounds checks for the zero halo, three
 * time buffers, no blocking, no fusion, no vector intrinsics.  OpenMP only
 * splits the outer x loop of the grid update.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_REAL_FLOAT
typedef float real;
#else
typedef double real;
#endif

enum { OR_OK = 0, OR_EINVAL = -1, OR_ERANGE = -3, OR_ENOMEM = -6 };

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int64_t shape[3];      /* 2D: (nx, nz); 3D: (nx, ny, nz); z fastest */
    double spacing[3];     /* metres per axis */
    int32_t order;         /* space order 2k (even, 2..16) */
    double dt;             /* seconds */
    int32_t nt;            /* number of time steps */
} oracle_grid;

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_real_bytes(void) { return (int)sizeof(real); }

/* ------------------------------------------------------------------------ */
/* Finite-difference weights of the central second derivative, order 2k.     */
/* Section "High-level API": f.dx2 at space_order=2 is (-2f + f(x-h) +       */
/* f(x+h))/h^2; higher orders use the 2k+1-point central stencil, whose      */
/* weights have the closed form                                              */
/*   c_j = 2 (-1)^(j+1) (k!)^2 / (j^2 (k-j)! (k+j)!),  j = 1..k              */
/*   c_0 = -2 sum_j c_j                                                      */
/* (c_{-j} = c_j).  Evaluated as a product of ratios, in double.             */
/* ------------------------------------------------------------------------ */
int oracle_fd_weights(int order, double *c)
{
    if (order < 2 || order > 16 || (order & 1) || !c) return OR_EINVAL;
    int k = order / 2;
    double s = 0.0;
    for (int j = 1; j <= k; ++j) {
        /* (k!)^2 / ((k-j)! (k+j)!) = prod_{i=1..j} (k-j+i) / (k+i) */
        double r = 1.0;
        for (int i = 1; i <= j; ++i) r *= (double)(k - j + i) / (double)(k + i);
        double cj = 2.0 * r / ((double)j * (double)j);
        if (!(j & 1)) cj = -cj;                 /* (-1)^(j+1) */
        c[j] = cj;
        s += cj;
    }
    c[0] = -2.0 * s;
    return OR_OK;
}

static int64_t npoints(const oracle_grid *g)
{
    int64_t n = 1;
    for (int a = 0; a < g->ndim; ++a) n *= g->shape[a];
    return n;
}

static int check_grid(const oracle_grid *g)
{
    if (!g || (g->ndim != 2 && g->ndim != 3)) return OR_EINVAL;
    for (int a = 0; a < g->ndim; ++a)
        if (g->shape[a] < 2 || !(g->spacing[a] > 0.0)) return OR_EINVAL;
    if (g->order < 2 || g->order > 16 || (g->order & 1)) return OR_EINVAL;
    if (!(g->dt > 0.0) || g->nt < 0) return OR_EINVAL;
    return OR_OK;
}

/* Zero outside the grid: the field is extended by zeros beyond its n points. */
static inline real at(const real *u, const int64_t *n, int ndim, int64_t i, int64_t j, int64_t k)
{
    if (ndim == 2) {               /* (i, k) = (x, z) */
        if (i < 0 || i >= n[0] || k < 0 || k >= n[1]) return (real)0;
        return u[i * n[1] + k];
    }
    if (i < 0 || i >= n[0] || j < 0 || j >= n[1] || k < 0 || k >= n[2]) return (real)0;
    return u[(i * n[1] + j) * n[2] + k];
}

/* (L u)_p = sum over axes a, sum over j = -k..k of c_|j| u(p + j e_a) / h_a^2 */
static real laplacian_at(const real *u, const int64_t *n, int ndim, const real *w,
                         const double *h, int k, int64_t i, int64_t j, int64_t l)
{
    real acc = 0;
    for (int a = 0; a < ndim; ++a) {
        real inv = (real)(1.0 / (h[a] * h[a]));
        real s = 0;
        for (int o = -k; o <= k; ++o) {
            real c = w[o < 0 ? -o : o];
            real v;
            if (ndim == 2) v = (a == 0) ? at(u, n, 2, i + o, 0, l) : at(u, n, 2, i, 0, l + o);
            else if (a == 0) v = at(u, n, 3, i + o, j, l);
            else if (a == 1) v = at(u, n, 3, i, j + o, l);
            else v = at(u, n, 3, i, j, l + o);
            s += c * v;
        }
        acc += s * inv;
    }
    return acc;
}

static void grid_dims(const oracle_grid *g, int64_t *n3)
{
    if (g->ndim == 2) { n3[0] = g->shape[0]; n3[1] = 1; n3[2] = g->shape[1]; }
    else { n3[0] = g->shape[0]; n3[1] = g->shape[1]; n3[2] = g->shape[2]; }
}

static void load_weights(int order, real *w)
{
    double c[9];
    oracle_fd_weights(order, c);
    for (int j = 0; j <= order / 2; ++j) w[j] = (real)c[j];
}

/* L u over the whole grid (exposed for operator tests). */
int oracle_laplacian(const oracle_grid *g, const double *u_in, double *out)
{
    int rc = check_grid(g);
    if (rc) return rc;
    int64_t N = npoints(g), n3[3];
    grid_dims(g, n3);
    real w[9];
    load_weights(g->order, w);
    real *u = (real *)malloc(sizeof(real) * N);
    if (!u) return OR_ENOMEM;
    for (int64_t p = 0; p < N; ++p) u[p] = (real)u_in[p];
    int k = g->order / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n3[0]; ++i)
        for (int64_t j = 0; j < n3[1]; ++j)
            for (int64_t l = 0; l < n3[2]; ++l)
                out[(i * n3[1] + j) * n3[2] + l] =
                    (double)laplacian_at(u, g->shape, g->ndim, w, g->spacing, k, i, j, l);
    free(u);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Sparse points (Section "Sparse point interpolation"): multilinear weights */
/* on the 2^d corners of the enclosing cell.  Per axis: x = p/h, i0 =        */
/* floor(x), i0 = n-2 on the upper edge, f = x - i0; corner c (bit a of c    */
/* selects i0+1 on axis a, axis 0 = most significant) has weight             */
/* prod_a (bit ? f_a : 1-f_a).  Coordinates outside [0, (n-1)h] (the upper   */
/* end evaluated as (n-1)*h in double) are ERANGE; x is capped at n-1 so a   */
/* point exactly on the upper edge cannot round past it.                     */
/* ------------------------------------------------------------------------ */
int oracle_sparse_weights(const oracle_grid *g, int npts, const double *coords,
                          int64_t *corner, double *weight)
{
    int rc = check_grid(g);
    if (rc) return rc;
    if (npts < 0 || (npts > 0 && (!coords || !corner || !weight))) return OR_EINVAL;
    int d = g->ndim, nc = 1 << d;
    for (int p = 0; p < npts; ++p) {
        int64_t i0[3];
        double f[3];
        for (int a = 0; a < d; ++a) {
            double c = coords[p * d + a];
            double top = (double)(g->shape[a] - 1) * g->spacing[a];
            if (!(c >= 0.0) || c > top) return OR_ERANGE;
            double x = c / g->spacing[a];
            if (x > (double)(g->shape[a] - 1)) x = (double)(g->shape[a] - 1);
            int64_t i = (int64_t)floor(x);
            if (i >= g->shape[a] - 1) i = g->shape[a] - 2;
            i0[a] = i;
            f[a] = x - (double)i;
        }
        for (int c = 0; c < nc; ++c) {
            int64_t flat = 0;
            double w = 1.0;
            for (int a = 0; a < d; ++a) {
                int bit = (c >> (d - 1 - a)) & 1;
                flat = flat * g->shape[a] + i0[a] + bit;
                w *= bit ? f[a] : 1.0 - f[a];
            }
            corner[(int64_t)p * nc + c] = flat;
            weight[(int64_t)p * nc + c] = w;
        }
    }
    return OR_OK;
}

typedef struct {
    int npts;
    int64_t *corner;  /* [npts][2^d] */
    real *w;          /* [npts][2^d] */
} sparse_set;

static int make_sparse(const oracle_grid *g, int npts, const double *coords, sparse_set *s)
{
    int nc = 1 << g->ndim;
    s->npts = npts;
    s->corner = NULL;
    s->w = NULL;
    if (npts <= 0) return OR_OK;
    s->corner = (int64_t *)malloc(sizeof(int64_t) * (size_t)npts * nc);
    double *wd = (double *)malloc(sizeof(double) * (size_t)npts * nc);
    s->w = (real *)malloc(sizeof(real) * (size_t)npts * nc);
    if (!s->corner || !wd || !s->w) { free(wd); return OR_ENOMEM; }
    int rc = oracle_sparse_weights(g, npts, coords, s->corner, wd);
    for (int64_t i = 0; i < (int64_t)npts * nc; ++i) s->w[i] = (real)wd[i];
    free(wd);
    return rc;
}

static void free_sparse(sparse_set *s) { free(s->corner); free(s->w); }

/* data[r] = sum_c w_{r,c} u[corner_{r,c}] */
static void sample(const sparse_set *s, int nc, const real *u, double *out)
{
    for (int p = 0; p < s->npts; ++p) {
        real acc = 0;
        for (int c = 0; c < nc; ++c) acc += s->w[p * nc + c] * u[s->corner[p * nc + c]];
        out[p] = (double)acc;
    }
}

/* u[corner_{s,c}] += dt^2 val_s w_{s,c} / a[corner], points in order, corners in order */
static void inject(const sparse_set *s, int nc, real dt2, const double *val,
                   const real *a, real *u)
{
    for (int p = 0; p < s->npts; ++p)
        for (int c = 0; c < nc; ++c) {
            int64_t i = s->corner[p * nc + c];
            u[i] += dt2 * (real)val[p] * s->w[p * nc + c] / a[i];
        }
}

/*
 * One time step of the solved update over every grid point:
 *   out = (2 m u - b u_other + dt^2 L u) / a
 * forward: u_other = u^{n-1}, out = u^{n+1};  adjoint: u_other = v^{k+1},
 * out = v^{k-1}.  Optional dense forcing adds dt^2 F / a.
 */
static void update(const oracle_grid *g, const real *w, const real *m, const real *a,
                   const real *b, const real *u, const real *u_other, real *out,
                   const real *force)
{
    int64_t n3[3];
    grid_dims(g, n3);
    int k = g->order / 2;
    real dt2 = (real)(g->dt * g->dt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n3[0]; ++i)
        for (int64_t j = 0; j < n3[1]; ++j)
            for (int64_t l = 0; l < n3[2]; ++l) {
                int64_t p = (i * n3[1] + j) * n3[2] + l;
                real lap = laplacian_at(u, g->shape, g->ndim, w, g->spacing, k, i, j, l);
                real num = (real)2 * m[p] * u[p] - b[p] * u_other[p] + dt2 * lap;
                if (force) num += dt2 * force[p];
                out[p] = num / a[p];
            }
}

typedef struct {
    real *m, *a, *b;
} coef;

static int make_coef(const oracle_grid *g, const double *m, const double *eta, coef *c)
{
    int64_t N = npoints(g);
    c->m = (real *)malloc(sizeof(real) * N);
    c->a = (real *)malloc(sizeof(real) * N);
    c->b = (real *)malloc(sizeof(real) * N);
    if (!c->m || !c->a || !c->b) return OR_ENOMEM;
    real hdt = (real)(0.5 * g->dt);
    for (int64_t p = 0; p < N; ++p) {
        real mm = (real)m[p], ee = eta ? (real)eta[p] : (real)0;
        c->m[p] = mm;
        c->a[p] = mm + ee * hdt;       /* m + eta dt/2 */
        c->b[p] = mm - ee * hdt;       /* m - eta dt/2 */
    }
    return OR_OK;
}

static void free_coef(coef *c) { free(c->m); free(c->a); free(c->b); }

/* Dense forcing at step n: F = sum_f T[n][f] P[f][:] (separable, test-only). */
static void dense_force(int64_t N, int nforce, const double *pat, const double *tco,
                        int n, real *F)
{
    for (int64_t p = 0; p < N; ++p) F[p] = 0;
    for (int f = 0; f < nforce; ++f) {
        real t = (real)tco[(int64_t)n * nforce + f];
        for (int64_t p = 0; p < N; ++p) F[p] += t * (real)pat[(int64_t)f * N + p];
    }
}

/*
 * Forward modelling (listing "lst:wave" with sources and receivers):
 *   for n = 0..nt-1:
 *     d[n][r] = sample of u^n at receiver r
 *     u^{n+1} = update(u^n, u^{n-1})   (+ dense forcing, test-only)
 *     u^{n+1}[corners of s] += dt^2 q[n][s] w / a
 * Start: u^{-1} = u^0 = 0, or the given (u_prev0, u0).
 * Outputs (each optional): d [nt][nrec], u_final = u^nt, u_prev_final =
 * u^{nt-1}, u_hist [nt+2][N] holding u^{-1}, u^0, ..., u^{nt}.
 */
int oracle_forward(const oracle_grid *g, const double *m, const double *eta,
                   int nsrc, const double *src_coords, const double *q,
                   int nrec, const double *rec_coords, double *d,
                   const double *u_prev0, const double *u0,
                   int nforce, const double *force_pat, const double *force_t,
                   double *u_final, double *u_prev_final, double *u_hist)
{
    int rc = check_grid(g);
    if (rc) return rc;
    if (!m || nsrc < 0 || nrec < 0 || (nsrc > 0 && !q) || (nrec > 0 && !d)) return OR_EINVAL;
    int64_t N = npoints(g);
    int nc = 1 << g->ndim;
    real w[9];
    load_weights(g->order, w);
    sparse_set S, R;
    coef C;
    memset(&C, 0, sizeof C);
    rc = make_sparse(g, nsrc, src_coords, &S);
    if (!rc) rc = make_sparse(g, nrec, rec_coords, &R);
    else R.corner = NULL, R.w = NULL;
    if (rc) { free_sparse(&S); free_sparse(&R); return rc; }
    rc = make_coef(g, m, eta, &C);
    real *u_m = (real *)calloc(N, sizeof(real));
    real *u_c = (real *)calloc(N, sizeof(real));
    real *u_p = (real *)calloc(N, sizeof(real));
    real *F = nforce > 0 ? (real *)malloc(sizeof(real) * N) : NULL;
    if (rc || !u_m || !u_c || !u_p || (nforce > 0 && !F)) {
        rc = OR_ENOMEM;
        goto out;
    }
    if (u_prev0) for (int64_t p = 0; p < N; ++p) u_m[p] = (real)u_prev0[p];
    if (u0) for (int64_t p = 0; p < N; ++p) u_c[p] = (real)u0[p];
    if (u_hist) {
        for (int64_t p = 0; p < N; ++p) u_hist[p] = (double)u_m[p];
        for (int64_t p = 0; p < N; ++p) u_hist[N + p] = (double)u_c[p];
    }
    real dt2 = (real)(g->dt * g->dt);
    for (int n = 0; n < g->nt; ++n) {
        if (nrec > 0) sample(&R, nc, u_c, d + (int64_t)n * nrec);
        if (F) dense_force(N, nforce, force_pat, force_t, n, F);
        update(g, w, C.m, C.a, C.b, u_c, u_m, u_p, F);
        if (nsrc > 0) inject(&S, nc, dt2, q + (int64_t)n * nsrc, C.a, u_p);
        real *t = u_m; u_m = u_c; u_c = u_p; u_p = t;
        if (u_hist) for (int64_t p = 0; p < N; ++p) u_hist[(int64_t)(n + 2) * N + p] = (double)u_c[p];
    }
    if (u_final) for (int64_t p = 0; p < N; ++p) u_final[p] = (double)u_c[p];
    if (u_prev_final) for (int64_t p = 0; p < N; ++p) u_prev_final[p] = (double)u_m[p];
out:
    free(u_m); free(u_c); free(u_p); free(F);
    free_coef(&C);
    free_sparse(&S); free_sparse(&R);
    return rc;
}

/*
 * Adjoint modelling (listing "lst:adjoint": minus eta u.dt, solved for the
 * backward time level), driven by receiver data and sampled at the sources:
 *   for k = nt-1..0:
 *     qadj[k][s] = sample of v^k at source s
 *     v^{k-1} = update(v^k, v^{k+1})
 *     v^{k-1}[corners of r] += dt^2 dres[k][r] w / a
 * Start v^{nt} = v^{nt-1} = 0.  This is the exact transpose of the forward
 * map q -> d above.  Optional v_hist [nt+1][N] holds v^0..v^{nt}.
 */
int oracle_adjoint(const oracle_grid *g, const double *m, const double *eta,
                   int nrec, const double *rec_coords, const double *dres,
                   int nsrc, const double *src_coords, double *qadj,
                   double *v_final, double *v_hist)
{
    int rc = check_grid(g);
    if (rc) return rc;
    if (!m || nsrc < 0 || nrec < 0 || (nrec > 0 && !dres) || (nsrc > 0 && !qadj)) return OR_EINVAL;
    int64_t N = npoints(g);
    int nc = 1 << g->ndim;
    real w[9];
    load_weights(g->order, w);
    sparse_set S, R;
    coef C;
    memset(&C, 0, sizeof C);
    rc = make_sparse(g, nsrc, src_coords, &S);
    if (!rc) rc = make_sparse(g, nrec, rec_coords, &R);
    else R.corner = NULL, R.w = NULL;
    if (rc) { free_sparse(&S); free_sparse(&R); return rc; }
    rc = make_coef(g, m, eta, &C);
    real *v_p = (real *)calloc(N, sizeof(real));   /* v^{k+1} */
    real *v_c = (real *)calloc(N, sizeof(real));   /* v^k */
    real *v_m = (real *)calloc(N, sizeof(real));   /* v^{k-1} */
    if (rc || !v_p || !v_c || !v_m) { rc = OR_ENOMEM; goto out; }
    real dt2 = (real)(g->dt * g->dt);
    if (v_hist) for (int64_t p = 0; p < N; ++p) v_hist[(int64_t)g->nt * N + p] = 0.0;
    for (int k = g->nt - 1; k >= 0; --k) {
        if (v_hist) for (int64_t p = 0; p < N; ++p) v_hist[(int64_t)k * N + p] = (double)v_c[p];
        if (nsrc > 0) sample(&S, nc, v_c, qadj + (int64_t)k * nsrc);
        update(g, w, C.m, C.a, C.b, v_c, v_p, v_m, NULL);
        if (nrec > 0) inject(&R, nc, dt2, dres + (int64_t)k * nrec, C.a, v_m);
        real *t = v_p; v_p = v_c; v_c = v_m; v_m = t;
    }
    /* after the k = 0 update v_p holds v^0, the last state sampled */
    if (v_final) for (int64_t p = 0; p < N; ++p) v_final[p] = (double)v_p[p];
out:
    free(v_p); free(v_c); free(v_m);
    free_coef(&C);
    free_sparse(&S); free_sparse(&R);
    return rc;
}

/*
 * Misfit and gradient with respect to m (eta held fixed) for one shot:
 *   J = 1/2 sum_n sum_r (d^n_r - dobs^n_r)^2
 *   g = -sum_{n=0}^{nt-1} v^n * (u^{n+1} - 2 u^n + u^{n-1}) / dt^2
 * with u from a fully stored forward run and v the adjoint driven by the
 * residual d - dobs.  grad_sbp (optional) receives the summation-by-parts
 * form -sum_n u^n * (v^{n+1} - 2 v^n + v^{n-1}) / dt^2, equal in exact
 * arithmetic because u^{-1} = u^0 = 0 and v^{nt} = v^{nt-1} = 0.
 * Memory: (nt + 2) N doubles for the stored forward.
 */
int oracle_gradient(const oracle_grid *g, const double *m, const double *eta,
                    int nsrc, const double *src_coords, const double *q,
                    int nrec, const double *rec_coords, const double *d_obs,
                    double *grad, double *grad_sbp, double *misfit, double *d_syn)
{
    int rc = check_grid(g);
    if (rc) return rc;
    if (!m || !grad || nrec <= 0 || !d_obs) return OR_EINVAL;
    int64_t N = npoints(g);
    int nt = g->nt;
    int nc = 1 << g->ndim;
    double *uh = (double *)malloc(sizeof(double) * (size_t)(nt + 2) * N);
    double *d = (double *)malloc(sizeof(double) * (size_t)nt * nrec);
    if (!uh || !d) { free(uh); free(d); return OR_ENOMEM; }
    rc = oracle_forward(g, m, eta, nsrc, src_coords, q, nrec, rec_coords, d,
                        NULL, NULL, 0, NULL, NULL, NULL, NULL, uh);
    if (rc) { free(uh); free(d); return rc; }
    /* residual and misfit */
    double J = 0.0;
    for (int64_t i = 0; i < (int64_t)nt * nrec; ++i) {
        double r = d[i] - d_obs[i];
        if (d_syn) d_syn[i] = d[i];
        d[i] = r;
        J += 0.5 * r * r;
    }
    if (misfit) *misfit = J;
    /* adjoint run with imaging */
    real w[9];
    load_weights(g->order, w);
    sparse_set R;
    coef C;
    memset(&C, 0, sizeof C);
    rc = make_sparse(g, nrec, rec_coords, &R);
    if (rc) { free_sparse(&R); free(uh); free(d); return rc; }
    rc = make_coef(g, m, eta, &C);
    real *v_p = (real *)calloc(N, sizeof(real));
    real *v_c = (real *)calloc(N, sizeof(real));
    real *v_m = (real *)calloc(N, sizeof(real));
    real *rd = (real *)malloc(sizeof(real) * (size_t)nt * nrec);
    if (rc || !v_p || !v_c || !v_m || !rd) { rc = OR_ENOMEM; goto out; }
    for (int64_t i = 0; i < (int64_t)nt * nrec; ++i) rd[i] = (real)d[i];
    for (int64_t p = 0; p < N; ++p) grad[p] = 0.0;
    if (grad_sbp) for (int64_t p = 0; p < N; ++p) grad_sbp[p] = 0.0;
    real dt2 = (real)(g->dt * g->dt);
    double idt2 = 1.0 / (g->dt * g->dt);
    (void)nc;
    for (int k = nt - 1; k >= 0; --k) {
        /* u^{k+1}, u^k, u^{k-1} live at uh[(k+2)N], uh[(k+1)N], uh[kN] */
        const double *un1 = uh + (int64_t)(k + 2) * N;
        const double *un0 = uh + (int64_t)(k + 1) * N;
        const double *unm = uh + (int64_t)k * N;
        for (int64_t p = 0; p < N; ++p)
            grad[p] -= (double)v_c[p] * (un1[p] - 2.0 * un0[p] + unm[p]) * idt2;
        update(g, w, C.m, C.a, C.b, v_c, v_p, v_m, NULL);
        for (int r = 0; r < nrec; ++r)
            for (int c = 0; c < nc; ++c) {
                int64_t i = R.corner[r * nc + c];
                v_m[i] += dt2 * rd[(int64_t)k * nrec + r] * R.w[r * nc + c] / C.a[i];
            }
        if (grad_sbp)
            for (int64_t p = 0; p < N; ++p)
                grad_sbp[p] -= un0[p] * ((double)v_p[p] - 2.0 * (double)v_c[p] + (double)v_m[p]) * idt2;
        real *t = v_p; v_p = v_c; v_c = v_m; v_m = t;
    }
out:
    free(v_p); free(v_c); free(v_m); free(rd);
    free_coef(&C);
    free_sparse(&R);
    free(uh); free(d);
    return rc;
}

/*
 * Diffusion (Section "2D Diffusion Example", equation "eqn:diffusion"),
 * forward Euler in time as in that section (time_order=1):
 *   u^{n+1} = u^n + dt a L u^n
 * with the same order-2k Laplacian and zero extension outside the grid.
 * a is the (possibly spatially varying) diffusion coefficient.
 */
int oracle_diffusion(const oracle_grid *g, const double *a_in, const double *u0, double *u_final)
{
    int rc = check_grid(g);
    if (rc) return rc;
    if (!a_in || !u0 || !u_final) return OR_EINVAL;
    int64_t N = npoints(g), n3[3];
    grid_dims(g, n3);
    int k = g->order / 2;
    real w[9];
    load_weights(g->order, w);
    real *u = (real *)malloc(sizeof(real) * N);
    real *v = (real *)malloc(sizeof(real) * N);
    real *a = (real *)malloc(sizeof(real) * N);
    if (!u || !v || !a) { free(u); free(v); free(a); return OR_ENOMEM; }
    for (int64_t p = 0; p < N; ++p) { u[p] = (real)u0[p]; a[p] = (real)a_in[p]; }
    real dt = (real)g->dt;
    for (int n = 0; n < g->nt; ++n) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n3[0]; ++i)
            for (int64_t j = 0; j < n3[1]; ++j)
                for (int64_t l = 0; l < n3[2]; ++l) {
                    int64_t p = (i * n3[1] + j) * n3[2] + l;
                    v[p] = u[p] + dt * a[p] * laplacian_at(u, g->shape, g->ndim, w, g->spacing, k, i, j, l);
                }
        real *t = u; u = v; v = t;
    }
    for (int64_t p = 0; p < N; ++p) u_final[p] = (double)u[p];
    free(u); free(v); free(a);
    return OR_OK;
}
