/*
 * fd6_oracle.c -- plain, slow FP64 CPU oracle for the sixth-order finite
 * difference right-hand side and the 2N-storage third-order Runge-Kutta
 * substep of Pekkila, Vaisala, Kapyla, Kapyla and Anjum (2017), "Methods for
 * compressible fluid simulation on GPUs using high-order finite differences".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the GPU library: every coefficient below is
 * written out here from the paper's equations.
 *
 * What it computes (paper section / equation):
 *   - ghost zone of R = 3 cells refreshed with periodic images
 *     (Sec. 4, opening paragraphs; the boundary step of Alg. 1-3)
 *   - first derivative, eq. (first_derivatives), Sec. 2.3
 *   - second derivative, eq. (second_derivatives), Sec. 2.3, with the
 *     prefactor read as 1/(180 dx^2) (the printed 1/(180 dx) is dimensionally
 *     wrong; the moment sum 2*(270 - 27*4 + 2*9) = 360 needs dx^2)
 *   - bidiagonal mixed derivative, eq. (mixed_derivatives), Sec. 2.3
 *   - continuity eq. (continuity), momentum eq. (navierstokes) and the
 *     traceless rate-of-strain tensor eq. (tensor), Sec. 2.1; D/Dt is the
 *     convective derivative, so d/dt = D/Dt - u.grad.  The external force f
 *     is zero unless orc_set_forcing gives one Fourier mode of eq. (forcing),
 *     Sec. 6, constant over a full step (the caller draws k, e and phi);
 *     grid point (i, j, k) sits at x = (i dx, j dy, k dz)
 *   - 2N-storage RK3, eq. (2N-RK_scheme) and Algorithm 1, Sec. 2.4.  The paper
 *     does not print alpha/beta beyond alpha(1) = 0; the values used are the
 *     Williamson (1980) low-storage RK3 coefficients
 *     alpha = (0, -5/9, -153/128), beta = (1/3, 15/16, 8/15).
 *   - the 19-point discretisation, Sec. 4.2 and Appendix A: grad div u as the
 *     first derivative of the (ghost-filled) divergence field; Algorithm 3
 *     splits its update into two passes, which in exact arithmetic equal the
 *     single update done here (the tests check the split against it)
 *
 * Storage: a field is a ghosted array of (nx+6)(ny+6)(nz+6) doubles with x
 * fastest; interior point (i,j,k) lives at ((k+3)(ny+6) + (j+3))(nx+6) + i+3.
 * Public entry points take compact nx*ny*nz arrays (x fastest) unless the
 * name says "ghosted".
 *
 * Arithmetic: FP64, no fused multiply-add (built without -mfma), operators
 * written in the mirrored-pair grouping of the printed stencils so that a
 * constant field has an exactly zero first derivative.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define R 3 /* stencil radius, Sec. 2.3: order n = 2R = 6 */

/* 2N-RK3 coefficients (see file header). */
static const double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

int orc_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nx, ny, nz;
    ptrdiff_t sx, sy, sz; /* strides of the ghosted layout */
} grid_t;

static grid_t make_grid(int nx, int ny, int nz) {
    grid_t g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.sx = 1;
    g.sy = nx + 2 * R;
    g.sz = (ptrdiff_t)(nx + 2 * R) * (ny + 2 * R);
    return g;
}

static size_t gsize(const grid_t *g) {
    return (size_t)(g->nx + 2 * R) * (g->ny + 2 * R) * (g->nz + 2 * R);
}

/* index of point (i,j,k), -R <= i < nx+R etc., in the ghosted layout */
static size_t gidx(const grid_t *g, int i, int j, int k) {
    return (size_t)((k + R) * g->sz + (j + R) * g->sy + (i + R));
}

static size_t cidx(const grid_t *g, int i, int j, int k) {
    return ((size_t)k * g->ny + j) * g->nx + i;
}

static int wrap(int i, int n) {
    int m = i % n;
    return m < 0 ? m + n : m;
}

/* Periodic boundary condition (Sec. 4): every ghost cell, faces, edges and
 * corners alike, receives the value of its periodic image in the
 * computational domain. */
void orc_fill_ghosts(int nx, int ny, int nz, double *f) {
    grid_t g = make_grid(nx, ny, nz);
    for (int k = -R; k < nz + R; ++k)
        for (int j = -R; j < ny + R; ++j)
            for (int i = -R; i < nx + R; ++i) {
                int inside = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                if (inside) continue;
                f[gidx(&g, i, j, k)] = f[gidx(&g, wrap(i, nx), wrap(j, ny), wrap(k, nz))];
            }
}

void orc_to_ghosted(int nx, int ny, int nz, const double *c, double *f) {
    grid_t g = make_grid(nx, ny, nz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) f[gidx(&g, i, j, k)] = c[cidx(&g, i, j, k)];
}

void orc_from_ghosted(int nx, int ny, int nz, const double *f, double *c) {
    grid_t g = make_grid(nx, ny, nz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) c[cidx(&g, i, j, k)] = f[gidx(&g, i, j, k)];
}

/* ------------------------------------------------------------------------ */
/* Finite-difference operators, Sec. 2.3                                     */
/* f: base pointer, c: centre index, s: stride along the axis, h: spacing.   */
/* ------------------------------------------------------------------------ */

/* eq. (first_derivatives): (-f[-3] + 9f[-2] - 45f[-1] + 45f[1] - 9f[2] + f[3]) / (60 h) */
static double op_d1(const double *f, size_t c, ptrdiff_t s, double h) {
    double num = 45.0 * (f[c + s] - f[c - s]) - 9.0 * (f[c + 2 * s] - f[c - 2 * s]) +
                 (f[c + 3 * s] - f[c - 3 * s]);
    return num / (60.0 * h);
}

/* eq. (second_derivatives): (2f[-3] - 27f[-2] + 270f[-1] - 490f[0] + 270f[1]
 * - 27f[2] + 2f[3]) / (180 h^2) */
static double op_d2(const double *f, size_t c, ptrdiff_t s, double h) {
    double num = 2.0 * (f[c - 3 * s] + f[c + 3 * s]) - 27.0 * (f[c - 2 * s] + f[c + 2 * s]) +
                 270.0 * (f[c - s] + f[c + s]) - 490.0 * f[c];
    return num / (180.0 * h * h);
}

/* eq. (mixed_derivatives): bidiagonal scheme along axes a and b,
 * sum_k w_k [f(+k,+k) - f(-k,+k) + f(-k,-k) - f(+k,-k)] / (720 ha hb),
 * w = (270, -27, 2) for k = 1, 2, 3. */
static double op_dmix(const double *f, size_t c, ptrdiff_t sa, ptrdiff_t sb, double ha,
                      double hb) {
    static const double w[3] = {270.0, -27.0, 2.0};
    double num = 0.0;
    for (int k = 1; k <= R; ++k) {
        double t = f[c + k * sa + k * sb] - f[c - k * sa + k * sb] + f[c - k * sa - k * sb] -
                   f[c + k * sa - k * sb];
        num += w[k - 1] * t;
    }
    return num / (720.0 * ha * hb);
}

/* Operator selector shared by the test entry point below. */
enum { OP_D1X, OP_D1Y, OP_D1Z, OP_D2X, OP_D2Y, OP_D2Z, OP_DXY, OP_DXZ, OP_DYZ };

static double apply_op(const double *f, size_t c, int op, ptrdiff_t sx, ptrdiff_t sy,
                       ptrdiff_t sz, double hx, double hy, double hz) {
    switch (op) {
    case OP_D1X: return op_d1(f, c, sx, hx);
    case OP_D1Y: return op_d1(f, c, sy, hy);
    case OP_D1Z: return op_d1(f, c, sz, hz);
    case OP_D2X: return op_d2(f, c, sx, hx);
    case OP_D2Y: return op_d2(f, c, sy, hy);
    case OP_D2Z: return op_d2(f, c, sz, hz);
    case OP_DXY: return op_dmix(f, c, sx, sy, hx, hy);
    case OP_DXZ: return op_dmix(f, c, sx, sz, hx, hz);
    case OP_DYZ: return op_dmix(f, c, sy, sz, hy, hz);
    default: return NAN;
    }
}

/* Apply one operator at every interior point of a ghosted array whose ghost
 * cells the caller has already filled (periodic or not).  out is compact. */
int orc_apply_op_ghosted(int nx, int ny, int nz, const double *f, int op, double hx, double hy,
                         double hz, double *out) {
    if (op < OP_D1X || op > OP_DYZ) return -1;
    grid_t g = make_grid(nx, ny, nz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                out[cidx(&g, i, j, k)] =
                    apply_op(f, gidx(&g, i, j, k), op, g.sx, g.sy, g.sz, hx, hy, hz);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side, Sec. 2.1                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double nu, cs, h[3];
} phys_t;

/* External force of eq. (navierstokes), one mode of eq. (forcing). */
static int g_force_on = 0;
static double g_force_k[3], g_force_a[3], g_force_phase;

/* Switches the force on for every later call: in = (kx, ky, kz, ex, ey, ez,
 * f0, phase, cs, dt).  Eq. (forcing): f(x) = Re{N f_k exp(i k.x + i phi)}
 * with N = f0 cs sqrt(|k| cs / dt) and f_k = (k x e) / sqrt(|k|^2 - (k.e)^2),
 * which is real, so f(x) = N f_k cos(k.x + phi).  NULL switches it off.
 * Returns -1 (force off) if e is parallel to k or |k| = 0. */
int orc_set_forcing(const double *in) {
    g_force_on = 0;
    if (!in) return 0;
    const double *k = in, *e = in + 3;
    const double f0 = in[6], phase = in[7], cs = in[8], dt = in[9];
    const double kk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    const double ke = k[0] * e[0] + k[1] * e[1] + k[2] * e[2];
    const double den2 = kk * kk - ke * ke;
    if (!(kk > 0.0) || !(den2 > 0.0) || !(dt > 0.0)) return -1;
    const double norm = f0 * cs * sqrt(kk * cs / dt);
    const double den = sqrt(den2);
    const double kxe[3] = {k[1] * e[2] - k[2] * e[1], k[2] * e[0] - k[0] * e[2],
                           k[0] * e[1] - k[1] * e[0]};
    for (int i = 0; i < 3; ++i) {
        g_force_k[i] = k[i];
        g_force_a[i] = norm * kxe[i] / den;
    }
    g_force_phase = phase;
    g_force_on = 1;
    return 0;
}

/* The amplitude vector N f_k in use (zeros when the force is off). */
void orc_get_forcing_amplitude(double a[3]) {
    for (int i = 0; i < 3; ++i) a[i] = g_force_on ? g_force_a[i] : 0.0;
}

typedef struct {
    const double *lnrho, *u[3];
    ptrdiff_t s[3]; /* strides along x, y, z */
} state_view_t;

/* Right-hand side at one point.  with_graddiv = 1 gives the full momentum
 * equation of the 55-point method (second derivatives by eq.
 * second_derivatives, mixed ones by eq. mixed_derivatives); with_graddiv = 0
 * drops the (nu/3) grad(div u) term, which is the first pass of the 19-point
 * method (Sec. 4.2).  Also returns div u from first derivatives. */
static void rhs_point(const state_view_t *v, size_t c, const phys_t *p, int with_graddiv,
                      const double xyz[3], double r[4], double *div_out) {
    double g[3], J[3][3], u[3];
    for (int j = 0; j < 3; ++j) g[j] = op_d1(v->lnrho, c, v->s[j], p->h[j]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = op_d1(v->u[i], c, v->s[j], p->h[j]); /* du_i/dx_j */
    for (int i = 0; i < 3; ++i) u[i] = v->u[i][c];
    double div = J[0][0] + J[1][1] + J[2][2];

    /* eq. (continuity): D lnrho / Dt = -div u */
    r[0] = -(u[0] * g[0] + u[1] * g[1] + u[2] * g[2]) - div;

    for (int i = 0; i < 3; ++i) {
        double adv = u[0] * J[i][0] + u[1] * J[i][1] + u[2] * J[i][2]; /* (u.grad) u_i */
        double lap = 0.0;                                               /* laplacian u_i */
        for (int j = 0; j < 3; ++j) lap += op_d2(v->u[i], c, v->s[j], p->h[j]);
        double sg = 0.0; /* (S . grad lnrho)_i with S from eq. (tensor) */
        for (int j = 0; j < 3; ++j) {
            double sij = 0.5 * (J[i][j] + J[j][i]) - (i == j ? div / 3.0 : 0.0);
            sg += sij * g[j];
        }
        double visc = lap + 2.0 * sg;
        if (with_graddiv) {
            double gd = 0.0; /* d_i (div u) = sum_j d_i d_j u_j */
            for (int j = 0; j < 3; ++j)
                gd += (i == j) ? op_d2(v->u[j], c, v->s[i], p->h[i])
                               : op_dmix(v->u[j], c, v->s[i], v->s[j], p->h[i], p->h[j]);
            visc += gd / 3.0;
        }
        /* eq. (navierstokes) */
        r[1 + i] = -adv - p->cs * p->cs * g[i] + p->nu * visc;
    }
    if (g_force_on) {
        const double arg = g_force_k[0] * xyz[0] + g_force_k[1] * xyz[1] +
                           g_force_k[2] * xyz[2] + g_force_phase;
        const double cphi = cos(arg);
        for (int i = 0; i < 3; ++i) r[1 + i] += g_force_a[i] * cphi;
    }
    if (div_out) *div_out = div;
}

enum { VAR_55P = 0, VAR_19P = 1 };

typedef struct {
    grid_t g;
    double *f[4]; /* ghosted lnrho, ux, uy, uz */
    double *w[4]; /* ghosted layout too (ghosts unused) */
    double *r[4]; /* right-hand side (ghosts unused) */
    double *d;    /* 19-point method: the divergence field, ghosted */
} box_t;

static void box_free(box_t *b) {
    for (int q = 0; q < 4; ++q) {
        free(b->f[q]);
        free(b->w[q]);
        free(b->r[q]);
    }
    free(b->d);
}

static int box_alloc(box_t *b, int nx, int ny, int nz) {
    memset(b, 0, sizeof(*b));
    b->g = make_grid(nx, ny, nz);
    size_t n = gsize(&b->g);
    for (int q = 0; q < 4; ++q) {
        b->f[q] = (double *)calloc(n, sizeof(double));
        b->w[q] = (double *)calloc(n, sizeof(double)); /* w = 0 at start */
        b->r[q] = (double *)calloc(n, sizeof(double));
        if (!b->f[q] || !b->w[q] || !b->r[q]) return -1;
    }
    b->d = (double *)calloc(n, sizeof(double));
    return b->d ? 0 : -1;
}

static state_view_t view_of(double *const f[4], const grid_t *g) {
    state_view_t v;
    v.lnrho = f[0];
    for (int i = 0; i < 3; ++i) v.u[i] = f[1 + i];
    v.s[0] = g->sx;
    v.s[1] = g->sy;
    v.s[2] = g->sz;
    return v;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Right-hand side d/dt (lnrho, u) of the periodic state b->f at every
 * interior point, into b->r.  55-point method: rhs_point with the grad div u
 * term of second and mixed derivatives.  19-point method (Sec. 4.2, Appendix
 * A): rhs_point without it, plus (nu/3) D1_i of the divergence field
 * d = D1 . u, whose ghost zone is filled with periodic images in between. */
static void rhs_all(box_t *b, const phys_t *p, int variant) {
    grid_t *g = &b->g;
    for (int q = 0; q < 4; ++q) orc_fill_ghosts(g->nx, g->ny, g->nz, b->f[q]);
    state_view_t v = view_of(b->f, g);
    const int full = variant == VAR_55P;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = gidx(g, i, j, k);
                const double xyz[3] = {i * p->h[0], j * p->h[1], k * p->h[2]};
                double r[4], div;
                rhs_point(&v, c, p, full, xyz, r, &div);
                b->d[c] = div;
                for (int q = 0; q < 4; ++q) b->r[q][c] = r[q];
            }
    if (full) return;
    orc_fill_ghosts(g->nx, g->ny, g->nz, b->d);
    const double nu3 = p->nu / 3.0;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = gidx(g, i, j, k);
                for (int q = 0; q < 3; ++q) b->r[1 + q][c] += nu3 * op_d1(b->d, c, v.s[q], p->h[q]);
            }
}

/* One substep s (0-based) of the 2N-storage RK3, eq. (2N-RK_scheme): the
 * right-hand side of the whole state first, then w <- alpha w + dt r and
 * state <- state + beta w at every point (the order of Algorithm 1, which
 * the in/out arrays of Algorithms 2 and 3 reproduce). */
static void substep(box_t *b, const phys_t *p, double dt, int s, int variant) {
    grid_t *g = &b->g;
    rhs_all(b, p, variant);
    const double a = RK_ALPHA[s], be = RK_BETA[s];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = gidx(g, i, j, k);
                for (int q = 0; q < 4; ++q) {
                    b->w[q][c] = a * b->w[q][c] + dt * b->r[q][c];
                    b->f[q][c] = b->f[q][c] + be * b->w[q][c];
                }
            }
}

static int check_dims(int nx, int ny, int nz) {
    return (nx >= 2 * R && ny >= 2 * R && nz >= 2 * R) ? 0 : -1;
}

/* Advance the compact fields by nsteps full RK3 steps (three substeps each),
 * in place.  variant 0 = 55-point, 1 = 19-point right-hand side.  w starts
 * at zero. */
int orc_rk3(int nx, int ny, int nz, double *lnrho, double *ux, double *uy, double *uz, double nu,
            double cs, double dx, double dy, double dz, double dt, int variant, int nsteps,
            int nthreads) {
    if (check_dims(nx, ny, nz) || (variant != VAR_55P && variant != VAR_19P) || nsteps < 0)
        return -1;
    set_threads(nthreads);
    box_t b;
    if (box_alloc(&b, nx, ny, nz)) {
        box_free(&b);
        return -2;
    }
    double *c[4] = {lnrho, ux, uy, uz};
    for (int q = 0; q < 4; ++q) orc_to_ghosted(nx, ny, nz, c[q], b.f[q]);
    phys_t p = {nu, cs, {dx, dy, dz}};
    for (int n = 0; n < nsteps; ++n)
        for (int s = 0; s < 3; ++s) substep(&b, &p, dt, s, variant);
    for (int q = 0; q < 4; ++q) orc_from_ghosted(nx, ny, nz, b.f[q], c[q]);
    box_free(&b);
    return 0;
}

/* Right-hand side d/dt (lnrho, ux, uy, uz) of the current compact state
 * (variant as for orc_rk3). */
int orc_rhs(int nx, int ny, int nz, const double *lnrho, const double *ux, const double *uy,
            const double *uz, double nu, double cs, double dx, double dy, double dz, int variant,
            double *r_lnrho, double *r_ux, double *r_uy, double *r_uz, int nthreads) {
    if (check_dims(nx, ny, nz) || (variant != VAR_55P && variant != VAR_19P)) return -1;
    set_threads(nthreads);
    box_t b;
    if (box_alloc(&b, nx, ny, nz)) {
        box_free(&b);
        return -2;
    }
    const double *c[4] = {lnrho, ux, uy, uz};
    double *out[4] = {r_lnrho, r_ux, r_uy, r_uz};
    for (int q = 0; q < 4; ++q) orc_to_ghosted(nx, ny, nz, c[q], b.f[q]);
    phys_t p = {nu, cs, {dx, dy, dz}};
    rhs_all(&b, &p, variant);
    for (int q = 0; q < 4; ++q) orc_from_ghosted(nx, ny, nz, b.r[q], out[q]);
    box_free(&b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local update of one point: the value after nsteps full steps at the       */
/* centre of a cubic patch, without any boundary condition.  Each substep    */
/* consumes R cells of the patch on every side (2R for the 19-point method,  */
/* whose grad div term differentiates the divergence field), so a patch      */
/* of half-width m = nsteps * 3 * R (55p) or nsteps * 6 * R (19p) determines  */
/* the centre exactly as the periodic run over the whole box does.  px, py,  */
/* pz: coordinates of the patch points along each axis (for the force).      */
/* ------------------------------------------------------------------------ */

int orc_rk3_patch(int m, const double *lnrho, const double *ux, const double *uy,
                  const double *uz, double nu, double cs, double dx, double dy, double dz,
                  double dt, int variant, int nsteps, const double *px, const double *py,
                  const double *pz, double out[4]) {
    const int shrink = (variant == VAR_55P) ? R : 2 * R;
    if (variant != VAR_55P && variant != VAR_19P) return -1;
    if (nsteps < 1 || m < 3 * shrink * nsteps) return -1;
    const int n = 2 * m + 1;
    const size_t nn = (size_t)n * n * n;
    double *f[4], *w[4], *r[4], *d;
    const double *in[4] = {lnrho, ux, uy, uz};
    int fail = 0;
    d = (double *)calloc(nn, sizeof(double));
    if (!d) fail = 1;
    for (int q = 0; q < 4; ++q) {
        f[q] = (double *)malloc(nn * sizeof(double));
        w[q] = (double *)calloc(nn, sizeof(double));
        r[q] = (double *)calloc(nn, sizeof(double));
        if (!f[q] || !w[q] || !r[q]) fail = 1;
        else memcpy(f[q], in[q], nn * sizeof(double));
    }
    if (!fail) {
        phys_t p = {nu, cs, {dx, dy, dz}};
        state_view_t v;
        v.s[0] = 1;
        v.s[1] = n;
        v.s[2] = (ptrdiff_t)n * n;
        const int full = variant == VAR_55P;
        int lo = 0; /* state is valid on [lo, n-lo)^3 */
        for (int step = 0; step < nsteps; ++step)
            for (int s = 0; s < 3; ++s) {
                const double a = RK_ALPHA[s], be = RK_BETA[s];
                v.lnrho = f[0];
                for (int i = 0; i < 3; ++i) v.u[i] = f[1 + i];
                /* the terms of rhs_point (and the divergence) where R cells
                 * of valid state surround the point */
                int a0 = lo + R, a1 = n - lo - R;
                for (int k = a0; k < a1; ++k)
                    for (int j = a0; j < a1; ++j)
                        for (int i = a0; i < a1; ++i) {
                            size_t c = ((size_t)k * n + j) * n + i;
                            const double xyz[3] = {px[i], py[j], pz[k]};
                            double rp[4], div;
                            rhs_point(&v, c, &p, full, xyz, rp, &div);
                            d[c] = div;
                            for (int q = 0; q < 4; ++q) r[q][c] = rp[q];
                        }
                if (!full) { /* (nu/3) D1_i d where R cells of d surround the point */
                    a0 += R;
                    a1 -= R;
                    const double nu3 = nu / 3.0;
                    for (int k = a0; k < a1; ++k)
                        for (int j = a0; j < a1; ++j)
                            for (int i = a0; i < a1; ++i) {
                                size_t c = ((size_t)k * n + j) * n + i;
                                for (int q = 0; q < 3; ++q)
                                    r[1 + q][c] += nu3 * op_d1(d, c, v.s[q], p.h[q]);
                            }
                }
                for (int k = a0; k < a1; ++k)
                    for (int j = a0; j < a1; ++j)
                        for (int i = a0; i < a1; ++i) {
                            size_t c = ((size_t)k * n + j) * n + i;
                            for (int q = 0; q < 4; ++q) {
                                w[q][c] = a * w[q][c] + dt * r[q][c];
                                f[q][c] = f[q][c] + be * w[q][c];
                            }
                        }
                lo += shrink;
            }
        size_t c = ((size_t)m * n + m) * n + m;
        for (int q = 0; q < 4; ++q) out[q] = f[q][c];
    }
    free(d);
    for (int q = 0; q < 4; ++q) {
        free(f[q]);
        free(w[q]);
        free(r[q]);
    }
    return fail ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Global diagnostics in FP64 (not part of the paper's kernels):             */
/* mass = dV sum exp(lnrho), kinetic energy = dV sum exp(lnrho) |u|^2 / 2,   */
/* sum lnrho, max |u|, and the number of points holding a non-finite value.  */
/* Sums are pairwise over the points in storage order.                       */
/* ------------------------------------------------------------------------ */

static double pairwise(const double *a, size_t n) {
    if (n <= 8) {
        double s = 0.0;
        for (size_t i = 0; i < n; ++i) s += a[i];
        return s;
    }
    size_t h = n / 2;
    return pairwise(a, h) + pairwise(a + h, n - h);
}

int orc_reduce(int nx, int ny, int nz, const double *lnrho, const double *ux, const double *uy,
               const double *uz, double dx, double dy, double dz, double out[5]) {
    size_t n = (size_t)nx * ny * nz;
    double *tm = (double *)malloc(n * sizeof(double));
    double *te = (double *)malloc(n * sizeof(double));
    if (!tm || !te) {
        free(tm);
        free(te);
        return -2;
    }
    double umax = 0.0;
    long long bad = 0;
    for (size_t i = 0; i < n; ++i) {
        double rho = exp(lnrho[i]);
        double u2 = ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i];
        tm[i] = rho;
        te[i] = 0.5 * rho * u2;
        double um = sqrt(u2);
        if (um > umax) umax = um;
        if (!isfinite(lnrho[i]) || !isfinite(ux[i]) || !isfinite(uy[i]) || !isfinite(uz[i])) ++bad;
    }
    double dv = dx * dy * dz;
    out[0] = dv * pairwise(tm, n);
    out[1] = dv * pairwise(te, n);
    out[2] = pairwise(lnrho, n);
    out[3] = umax;
    out[4] = (double)bad;
    free(tm);
    free(te);
    return 0;
}
