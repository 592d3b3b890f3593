/*
 * FP64 CPU oracle for the high-order stencil sweep and the acoustic wave step
 * it drives (MMStencil, arXiv 2507.11067).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * HIP library is checked against.  It shares no code, header or table with the
 * library; only the test suite, the smoke check and the benchmark's CPU
 * baseline load it.
 *
 * Every routine is a direct loop over the definition, in double precision,
 * with OpenMP only over the outermost (z) loop of a sweep.  Grids use the
 * padded layout: interior point (z, y, x) sits at element
 *   (z + H) * sz + (y + H) * sy + (x + H)
 * and the halo cells are read as stored (zero for the workloads).
 *
 * Passages followed:
 *  - star and box stencils: the problem statement of Sec. I (star reaches
 *    neighbours along the axes only, box reaches the whole (2r+1)^d cube) and
 *    the radius-4 / 8th-order high-order case of Sec. II-A; the 2-D kernels of
 *    Table I (2DStar, 2DBox) applied to every z-plane of a stack of planes;
 *  - the acoustic time step: the second-order-in-time wave update that RTM
 *    (Sec. II-A, Sec. V-F) is built on, u^{n+1} = 2u^n - u^{n-1} + v^2 dt^2 L u^n
 *    + source, with the damping sponge, source and receiver reading listed in
 *    the design notes;
 *  - the adjoint step and the gradient: the exact transpose of that recurrence
 *    (derived in the design notes; the paper has no adjoint);
 *  - the VTI and TTI pseudo-acoustic pairs of Sec. II-A, with the mixed second
 *    derivatives of the TTI operators composed from first-derivative stencils
 *    (Sec. IV-G).
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    long nx, ny, nz; /* interior extent */
    long H;          /* halo width */
    long sy, sz;     /* element strides of y and z; x stride is 1 */
} orc_grid;

static inline long at(const orc_grid *g, long z, long y, long x) {
    return (z + g->H) * g->sz + (y + g->H) * g->sy + (x + g->H);
}

/* Star stencil, plain definition.
 * out(p) = sum_{a in z,y,x} sum_{k=-r..r} c[a][k+r] * in(p + k e_a)
 * c is [3][2r+1]: axis z first, then y, then x. */
void orc_star(const double *in, double *out, const orc_grid *g, int r, const double *c) {
    const int w = 2 * r + 1;
    const double *cz = c, *cy = c + w, *cx = c + 2 * w;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                double s = 0.0;
                for (int k = -r; k <= r; ++k) s += cz[k + r] * in[at(g, z + k, y, x)];
                for (int k = -r; k <= r; ++k) s += cy[k + r] * in[at(g, z, y + k, x)];
                for (int k = -r; k <= r; ++k) s += cx[k + r] * in[at(g, z, y, x + k)];
                out[at(g, z, y, x)] = s;
            }
}

/* Box stencil, plain definition.
 * out(p) = sum_{dz,dy,dx in [-r,r]} c[dz+r][dy+r][dx+r] * in(p + (dz,dy,dx)) */
void orc_box(const double *in, double *out, const orc_grid *g, int r, const double *c) {
    const int w = 2 * r + 1;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                double s = 0.0;
                for (int dz = -r; dz <= r; ++dz)
                    for (int dy = -r; dy <= r; ++dy)
                        for (int dx = -r; dx <= r; ++dx)
                            s += c[((dz + r) * w + (dy + r)) * w + (dx + r)] *
                                 in[at(g, z + dz, y + dy, x + dx)];
                out[at(g, z, y, x)] = s;
            }
}

/* The same two definitions evaluated at a list of interior points only
 * (pts holds npts (z, y, x) triples); used to check sampled outputs of large
 * grids without sweeping the whole grid. */
void orc_star_at(const double *in, const orc_grid *g, int r, const double *c, long npts,
                 const long *pts, double *out) {
    const int w = 2 * r + 1;
    const double *cz = c, *cy = c + w, *cx = c + 2 * w;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < npts; ++i) {
        const long z = pts[3 * i], y = pts[3 * i + 1], x = pts[3 * i + 2];
        double s = 0.0;
        for (int k = -r; k <= r; ++k) s += cz[k + r] * in[at(g, z + k, y, x)];
        for (int k = -r; k <= r; ++k) s += cy[k + r] * in[at(g, z, y + k, x)];
        for (int k = -r; k <= r; ++k) s += cx[k + r] * in[at(g, z, y, x + k)];
        out[i] = s;
    }
}

void orc_box_at(const double *in, const orc_grid *g, int r, const double *c, long npts,
                const long *pts, double *out) {
    const int w = 2 * r + 1;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < npts; ++i) {
        const long z = pts[3 * i], y = pts[3 * i + 1], x = pts[3 * i + 2];
        double s = 0.0;
        for (int dz = -r; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx)
                    s += c[((dz + r) * w + (dy + r)) * w + (dx + r)] *
                         in[at(g, z + dz, y + dy, x + dx)];
        out[i] = s;
    }
}

/* 2-D star on every z-plane of the stack (Table I, 2DStarR2 / 2DStarR4):
 * out(z, y, x) = sum_{k=-r..r} cy[k+r] in(z, y+k, x) + sum_{k=-r..r} cx[k+r] in(z, y, x+k)
 * c is [2][2r+1]: axis y, then x.  No z neighbour is read. */
static double star2d_at(const double *in, const orc_grid *g, int r, const double *c, long z,
                        long y, long x) {
    const int w = 2 * r + 1;
    const double *cy = c, *cx = c + w;
    double s = 0.0;
    for (int k = -r; k <= r; ++k) s += cy[k + r] * in[at(g, z, y + k, x)];
    for (int k = -r; k <= r; ++k) s += cx[k + r] * in[at(g, z, y, x + k)];
    return s;
}

/* 2-D box on every z-plane (Table I, 2DBoxR2 / 2DBoxR3):
 * out(z, y, x) = sum_{dy,dx in [-r,r]} c[dy+r][dx+r] in(z, y+dy, x+dx) */
static double box2d_at(const double *in, const orc_grid *g, int r, const double *c, long z,
                       long y, long x) {
    const int w = 2 * r + 1;
    double s = 0.0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) s += c[(dy + r) * w + (dx + r)] * in[at(g, z, y + dy, x + dx)];
    return s;
}

void orc_star2d(const double *in, double *out, const orc_grid *g, int r, const double *c) {
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) out[at(g, z, y, x)] = star2d_at(in, g, r, c, z, y, x);
}

void orc_box2d(const double *in, double *out, const orc_grid *g, int r, const double *c) {
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) out[at(g, z, y, x)] = box2d_at(in, g, r, c, z, y, x);
}

void orc_star2d_at(const double *in, const orc_grid *g, int r, const double *c, long npts,
                   const long *pts, double *out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < npts; ++i)
        out[i] = star2d_at(in, g, r, c, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
}

void orc_box2d_at(const double *in, const orc_grid *g, int r, const double *c, long npts,
                  const long *pts, double *out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < npts; ++i)
        out[i] = box2d_at(in, g, r, c, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
}

/* Transpose of the star operator on the interior (zero outside it):
 * out(q) = sum_{a,k} c[a][k+r] * in(q - k e_a), with in read as 0 off the interior. */
static void star_transpose(const double *in, double *out, const orc_grid *g, int r,
                           const double *c) {
    const int w = 2 * r + 1;
    const double *cs[3] = {c, c + w, c + 2 * w};
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int k = -r; k <= r; ++k) {
                        long zz = z - (a == 0 ? k : 0);
                        long yy = y - (a == 1 ? k : 0);
                        long xx = x - (a == 2 ? k : 0);
                        if (zz < 0 || zz >= g->nz || yy < 0 || yy >= g->ny || xx < 0 || xx >= g->nx)
                            continue;
                        s += cs[a][k + r] * in[at(g, zz, yy, xx)];
                    }
                out[at(g, z, y, x)] = s;
            }
}

/* One-dimensional damping profile of the absorbing sponge.  Cell i of n is at
 * distance d from the nearest damped face (d = i from the low face, n-1-i from
 * the high face); inside the layer (d < W) the factor is exp(-(alpha (W - d))^2),
 * elsewhere 1. */
void orc_sponge_1d(long n, int W, double alpha, int damp_lo, int damp_hi, double *g) {
    for (long i = 0; i < n; ++i) {
        double f = 1.0;
        if (damp_lo && i < W) f *= exp(-pow(alpha * (double)(W - i), 2.0));
        long j = n - 1 - i;
        if (damp_hi && j < W) f *= exp(-pow(alpha * (double)(W - j), 2.0));
        g[i] = f;
    }
}

typedef struct {
    orc_grid g;
    int r;
    const double *lap;    /* r+1 per-axis weights at unit spacing: centre, k = 1..r */
    const double *c2;     /* padded: (v dt / h)^2 */
    int sponge_width;
    double sponge_alpha;
    int sponge_faces;     /* 1 x-lo, 2 x-hi, 4 y-lo, 8 y-hi, 16 z-lo, 32 z-hi */
    long src_z, src_y, src_x;
    const double *src;    /* [nt]: dt^2 f(n dt) */
    int nt;
} orc_wave;

/* Full-grid damping factor G(z,y,x) = gz(z) gy(y) gx(x), interior only. */
static double *sponge_field(const orc_wave *w) {
    const orc_grid *g = &w->g;
    double *gx = malloc(sizeof(double) * g->nx);
    double *gy = malloc(sizeof(double) * g->ny);
    double *gz = malloc(sizeof(double) * g->nz);
    orc_sponge_1d(g->nx, w->sponge_width, w->sponge_alpha, w->sponge_faces & 1, w->sponge_faces & 2, gx);
    orc_sponge_1d(g->ny, w->sponge_width, w->sponge_alpha, w->sponge_faces & 4, w->sponge_faces & 8, gy);
    orc_sponge_1d(g->nz, w->sponge_width, w->sponge_alpha, w->sponge_faces & 16, w->sponge_faces & 32, gz);
    double *G = calloc((size_t)(g->nz + 2 * g->H) * g->sz, sizeof(double));
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) G[at(g, z, y, x)] = gz[z] * gy[y] * gx[x];
    free(gx); free(gy); free(gz);
    return G;
}

static void lap_table(const orc_wave *w, double *c) {
    const int r = w->r, n = 2 * r + 1;
    for (int a = 0; a < 3; ++a)
        for (int k = -r; k <= r; ++k) c[a * n + k + r] = w->lap[k < 0 ? -k : k];
}

static size_t field_len(const orc_grid *g) { return (size_t)(g->nz + 2 * g->H) * g->sz; }

/* One forward step n (1 <= n < nt), G given:
 *   u^{n+1} = G (2 u^n - G u^{n-1} + C2 S u^n) + dt^2 f^n delta_src
 * Also records the receiver plane d^n = u^n(z = 0) into trace (ny*nx) and adds
 * (u^{n+1})^2 to image when those are non-NULL. */
static void step_with_G(const orc_wave *w, const double *G, const double *lapc, int n,
                        const double *uprev, const double *ucur, double *unext,
                        double *trace, double *image, double *work) {
    const orc_grid *g = &w->g;
    orc_star(ucur, work, g, w->r, lapc);
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                long i = at(g, z, y, x);
                unext[i] = G[i] * (2.0 * ucur[i] - G[i] * uprev[i] + w->c2[i] * work[i]);
            }
    if (n >= 0 && n < w->nt) unext[at(g, w->src_z, w->src_y, w->src_x)] += w->src[n];
    if (trace)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) trace[y * g->nx + x] = ucur[at(g, 0, y, x)];
    if (image)
        for (long z = 0; z < g->nz; ++z)
            for (long y = 0; y < g->ny; ++y)
                for (long x = 0; x < g->nx; ++x) {
                    long i = at(g, z, y, x);
                    image[i] += unext[i] * unext[i];
                }
}

void orc_wave_step(const orc_wave *w, int n, const double *uprev, const double *ucur,
                   double *unext, double *trace, double *image) {
    double *G = sponge_field(w);
    double lapc[27];
    lap_table(w, lapc);
    double *work = calloc(field_len(&w->g), sizeof(double));
    step_with_G(w, G, lapc, n, uprev, ucur, unext, trace, image, work);
    free(work); free(G);
}

/* Forward run.  Inputs u^0, u^1; steps n = 1..nt-1 produce u^2..u^nt.
 * traces: [nt][ny][nx], d^n = u^n(z = 0) for n = 0..nt-1.
 * states: NULL, or (nt+1) padded fields receiving u^0..u^nt.
 * last:   NULL, or 2 padded fields receiving u^{nt-1}, u^nt.
 * image:  NULL, or a padded field that accumulates sum_n (u^{n+1})^2. */
void orc_wave_forward(const orc_wave *w, const double *u0, const double *u1, double *traces,
                      double *states, double *last, double *image) {
    const orc_grid *g = &w->g;
    const size_t L = field_len(g);
    double *G = sponge_field(w);
    double lapc[27];
    lap_table(w, lapc);
    double *a = malloc(L * sizeof(double)), *b = malloc(L * sizeof(double));
    double *c = calloc(L, sizeof(double)), *work = calloc(L, sizeof(double));
    memcpy(a, u0, L * sizeof(double));
    memcpy(b, u1, L * sizeof(double));
    for (long y = 0; y < g->ny; ++y)
        for (long x = 0; x < g->nx; ++x) traces[y * g->nx + x] = a[at(g, 0, y, x)];
    if (states) {
        memcpy(states, a, L * sizeof(double));
        memcpy(states + L, b, L * sizeof(double));
    }
    for (int n = 1; n < w->nt; ++n) {
        double *tr = traces + (size_t)n * g->ny * g->nx;
        step_with_G(w, G, lapc, n, a, b, c, tr, image, work);
        double *t = a; a = b; b = c; c = t;  /* a = u^n, b = u^{n+1} */
        if (states) memcpy(states + (size_t)(n + 1) * L, b, L * sizeof(double));
    }
    if (last) {
        memcpy(last, a, L * sizeof(double));
        memcpy(last + L, b, L * sizeof(double));
    }
    free(a); free(b); free(c); free(work); free(G);
}

/* One adjoint step n, G given.  For n >= 1:
 *   lam^n = 2 G lam^{n+1} - G^2 lam^{n+2} + S^T (C2 G lam^{n+1}) + R^T r^n
 *   grad_c2 += G lam^{n+1} S u^n
 * For n = 0 (u^0 enters only through the G^2 term of step 1 and the receivers):
 *   lam^0 = -G^2 lam^2 + R^T r^0. */
static void adjoint_with_G(const orc_wave *w, const double *G, const double *lapc, int n,
                           const double *lam2, const double *lam1, double *lam0,
                           const double *resid, const double *un, double *grad,
                           double *work, double *work2) {
    const orc_grid *g = &w->g;
    if (n >= 1) {
#pragma omp parallel for schedule(static)
        for (long z = 0; z < g->nz; ++z)
            for (long y = 0; y < g->ny; ++y)
                for (long x = 0; x < g->nx; ++x) {
                    long i = at(g, z, y, x);
                    work[i] = w->c2[i] * G[i] * lam1[i];
                }
        star_transpose(work, work2, g, w->r, lapc);
        if (grad) orc_star(un, work, g, w->r, lapc);
    }
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                long i = at(g, z, y, x);
                double v = -G[i] * G[i] * lam2[i];
                if (n >= 1) {
                    v += 2.0 * G[i] * lam1[i] + work2[i];
                    if (grad) grad[i] += G[i] * lam1[i] * work[i];
                }
                lam0[i] = v;
            }
    if (resid)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) lam0[at(g, 0, y, x)] += resid[y * g->nx + x];
}

void orc_adjoint_step(const orc_wave *w, int n, const double *lam2, const double *lam1,
                      double *lam0, const double *resid, const double *un, double *grad) {
    const size_t L = field_len(&w->g);
    double *G = sponge_field(w);
    double lapc[27];
    lap_table(w, lapc);
    double *work = calloc(L, sizeof(double)), *work2 = calloc(L, sizeof(double));
    adjoint_with_G(w, G, lapc, n, lam2, lam1, lam0, resid, un, grad, work, work2);
    free(work); free(work2); free(G);
}

/* Full adjoint run over stored forward states u^0..u^nt (only u^1..u^{nt-1} are
 * read).  resid: [nt][ny][nx] = d - d_obs.  Outputs: grad_c2 (padded, overwritten),
 * lam0 = dJ/du^0, lam1 = dJ/du^1, and, if grad_src is non-NULL, dJ/d(dt^2 f^n)
 * = lam^{n+1}(src) for n = 1..nt-1 (lam^nt = 0; f^0 is unused, its entry is 0). */
void orc_wave_adjoint(const orc_wave *w, const double *states, const double *resid,
                      double *grad_c2, double *lam0_out, double *lam1_out, double *grad_src) {
    const orc_grid *g = &w->g;
    const size_t L = field_len(g);
    const size_t P = (size_t)g->ny * g->nx;
    double *G = sponge_field(w);
    double lapc[27];
    lap_table(w, lapc);
    double *l2 = calloc(L, sizeof(double)), *l1 = calloc(L, sizeof(double));
    double *l0 = calloc(L, sizeof(double));
    double *work = calloc(L, sizeof(double)), *work2 = calloc(L, sizeof(double));
    memset(grad_c2, 0, L * sizeof(double));
    const long isrc = at(g, w->src_z, w->src_y, w->src_x);
    if (grad_src) {
        grad_src[0] = 0.0;          /* f^0 is never injected: u^1 is an input */
        grad_src[w->nt - 1] = 0.0;  /* lam^nt = 0 */
    }
    for (int n = w->nt - 1; n >= 0; --n) {
        adjoint_with_G(w, G, lapc, n, l2, l1, l0, resid + (size_t)n * P,
                       n >= 1 ? states + (size_t)n * L : NULL, grad_c2, work, work2);
        if (grad_src && n >= 2) grad_src[n - 1] = l0[isrc];
        double *t = l2; l2 = l1; l1 = l0; l0 = t;  /* l1 = lam^n, l2 = lam^{n+1} */
        if (n == 1) memcpy(lam1_out, l1, L * sizeof(double));
    }
    memcpy(lam0_out, l1, L * sizeof(double));
    free(l2); free(l1); free(l0); free(work); free(work2); free(G);
}

/* VTI pair.  Sec. II-A prints a sigma_H / sigma_V system whose second equation
 * swaps the fields (as printed, the difference sigma_H - sigma_V obeys
 * D_tt = v^2 (D_xx + D_yy - D_zz), which is ill-posed).  The TTI system printed
 * right after it reduces, for zero tilt (H1 = d_zz, H2 = d_xx + d_yy), zero shear
 * velocity and alpha = sqrt(1 + 2 delta), to the well-posed pseudo-acoustic pair
 * used here, with a = 1 + 2 epsilon and b = sqrt(1 + 2 delta) given as fields:
 *   H^{n+1} = G (2 H^n - G H^{n-1} + C2 (a Sxy H^n + b Szz V^n)) + dt^2 f^n delta_src
 *   V^{n+1} = G (2 V^n - G V^{n-1} + C2 (b Sxy H^n +   Szz V^n)) + dt^2 f^n delta_src
 * Sxy = Sxx + Syy and Szz are the axis parts of the star with weights lap; the
 * leapfrog, sponge and source are those of the acoustic step.  The receiver plane
 * records H^n(z = 0). */
static void axis_tables(const orc_wave *w, double *cxy, double *cz) {
    const int r = w->r, n = 2 * r + 1;
    for (int k = -r; k <= r; ++k) {
        const double v = w->lap[k < 0 ? -k : k];
        cxy[0 * n + k + r] = 0.0;  cxy[1 * n + k + r] = v;  cxy[2 * n + k + r] = v;
        cz[0 * n + k + r] = v;     cz[1 * n + k + r] = 0.0; cz[2 * n + k + r] = 0.0;
    }
}

static void vti_step_with_G(const orc_wave *w, const double *G, int n, const double *a,
                            const double *b, const double *hp, const double *hc, double *hn,
                            const double *vp, const double *vc, double *vn, double *trace,
                            double *w1, double *w2, double *w3, double *w4) {
    const orc_grid *g = &w->g;
    double cxy[27], cz[27];
    axis_tables(w, cxy, cz);
    orc_star(hc, w1, g, w->r, cxy);  /* Sxy H */
    orc_star(vc, w2, g, w->r, cz);   /* Szz V */
    (void)w3; (void)w4;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                long i = at(g, z, y, x);
                hn[i] = G[i] * (2.0 * hc[i] - G[i] * hp[i] + w->c2[i] * (a[i] * w1[i] + b[i] * w2[i]));
                vn[i] = G[i] * (2.0 * vc[i] - G[i] * vp[i] + w->c2[i] * (b[i] * w1[i] + w2[i]));
            }
    if (n >= 0 && n < w->nt) {
        const long s = at(g, w->src_z, w->src_y, w->src_x);
        hn[s] += w->src[n];
        vn[s] += w->src[n];
    }
    if (trace)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) trace[y * g->nx + x] = hc[at(g, 0, y, x)];
}

void orc_vti_step(const orc_wave *w, int n, const double *a, const double *b, const double *hp,
                  const double *hc, double *hn, const double *vp, const double *vc, double *vn,
                  double *trace) {
    const size_t L = field_len(&w->g);
    double *G = sponge_field(w);
    double *w1 = calloc(L, sizeof(double)), *w2 = calloc(L, sizeof(double));
    double *w3 = calloc(L, sizeof(double)), *w4 = calloc(L, sizeof(double));
    vti_step_with_G(w, G, n, a, b, hp, hc, hn, vp, vc, vn, trace, w1, w2, w3, w4);
    free(w1); free(w2); free(w3); free(w4); free(G);
}

/* Forward VTI run from (H^0, H^1, V^0, V^1); traces [nt][ny][nx] of H; last receives
 * H^{nt-1}, H^nt, V^{nt-1}, V^nt (4 padded fields) when non-NULL. */
void orc_vti_forward(const orc_wave *w, const double *a, const double *b, const double *h0,
                     const double *h1, const double *v0, const double *v1, double *traces,
                     double *last) {
    const orc_grid *g = &w->g;
    const size_t L = field_len(g);
    double *G = sponge_field(w);
    double *H[3], *V[3];
    for (int i = 0; i < 3; ++i) {
        H[i] = calloc(L, sizeof(double));
        V[i] = calloc(L, sizeof(double));
    }
    double *w1 = calloc(L, sizeof(double)), *w2 = calloc(L, sizeof(double));
    double *w3 = calloc(L, sizeof(double)), *w4 = calloc(L, sizeof(double));
    memcpy(H[0], h0, L * sizeof(double)); memcpy(H[1], h1, L * sizeof(double));
    memcpy(V[0], v0, L * sizeof(double)); memcpy(V[1], v1, L * sizeof(double));
    for (long y = 0; y < g->ny; ++y)
        for (long x = 0; x < g->nx; ++x) traces[y * g->nx + x] = h0[at(g, 0, y, x)];
    for (int n = 1; n < w->nt; ++n) {
        double *tr = traces + (size_t)n * g->ny * g->nx;
        vti_step_with_G(w, G, n, a, b, H[(n - 1) % 3], H[n % 3], H[(n + 1) % 3],
                        V[(n - 1) % 3], V[n % 3], V[(n + 1) % 3], tr, w1, w2, w3, w4);
    }
    if (last) {
        const int m = w->nt;
        memcpy(last, H[(m - 1) % 3], L * sizeof(double));
        memcpy(last + L, H[m % 3], L * sizeof(double));
        memcpy(last + 2 * L, V[(m - 1) % 3], L * sizeof(double));
        memcpy(last + 3 * L, V[m % 3], L * sizeof(double));
    }
    for (int i = 0; i < 3; ++i) { free(H[i]); free(V[i]); }
    free(w1); free(w2); free(w3); free(w4); free(G);
}

/* ------------------------------------------------------------------ TTI
 * Pseudo-acoustic TTI pair (Sec. II-A), in units of C2 = (v_pz dt / h)^2:
 *   p'' = C2 [ (1+2eps) H2 p + alpha H1 q + sigma H1 (p - alpha q) ]
 *   q'' = C2 [ ((1+2delta)/alpha) H2 p + H1 q - sigma H2 (p/alpha - q) ]
 * with v_px^2 = (1+2eps) v_pz^2, v_pn^2 = (1+2delta) v_pz^2, sigma = v_sz^2 / v_pz^2,
 *   H1 = st^2 cp^2 Dxx + st^2 sp^2 Dyy + ct^2 Dzz + st^2 sin(2phi) Dxy
 *        + sin(2theta) sp Dyz + sin(2theta) cp Dxz      (st = sin theta, cp = cos phi ...)
 *   H2 = Dxx + Dyy + Dzz - H1.
 * Second derivatives along an axis are the per-axis star weights; a mixed
 * derivative Da Db is the product of two first-derivative stencils
 * D f(i) = sum_{k=1..r} d_k (f(i+k) - f(i-k)), i.e. the 2-D stencil with weights
 * d_i d_j on the plane of the two axes (Sec. IV-G builds it by composing the two
 * one-dimensional stencils).  Grid values are read as stored (halo included). */
typedef struct {
    const double *eps, *delta, *theta, *phi; /* padded fields */
    double sigma;                            /* v_sz^2 / v_pz^2 */
    double alpha;                            /* coupling scale of q */
    const double *d1;                        /* first-derivative weights d_1..d_r */
} orc_tti;

static double axis_d2(const double *f, const orc_grid *g, const double *lap, int r, long z, long y,
                      long x, int az, int ay, int ax) {
    double s = lap[0] * f[at(g, z, y, x)];
    for (int k = 1; k <= r; ++k)
        s += lap[k] * (f[at(g, z + k * az, y + k * ay, x + k * ax)] +
                       f[at(g, z - k * az, y - k * ay, x - k * ax)]);
    return s;
}

/* Da Db f with a = (az, ay, ax), b = (bz, by, bx) unit axis vectors */
static double mixed_d2(const double *f, const orc_grid *g, const double *d1, int r, long z, long y,
                       long x, const int *a, const int *b) {
    double s = 0.0;
    for (int i = 1; i <= r; ++i)
        for (int j = 1; j <= r; ++j) {
            const double pp = f[at(g, z + i * a[0] + j * b[0], y + i * a[1] + j * b[1], x + i * a[2] + j * b[2])];
            const double pm = f[at(g, z + i * a[0] - j * b[0], y + i * a[1] - j * b[1], x + i * a[2] - j * b[2])];
            const double mp = f[at(g, z - i * a[0] + j * b[0], y - i * a[1] + j * b[1], x - i * a[2] + j * b[2])];
            const double mm = f[at(g, z - i * a[0] - j * b[0], y - i * a[1] - j * b[1], x - i * a[2] - j * b[2])];
            s += d1[i - 1] * d1[j - 1] * (pp - pm - mp + mm);
        }
    return s;
}

/* (L f, H1 f) at one interior point; L = Dxx + Dyy + Dzz */
static void tti_ops(const orc_wave *w, const orc_tti *t, const double *f, long z, long y, long x,
                    double *lf, double *h1f) {
    static const int EX[3] = {0, 0, 1}, EY[3] = {0, 1, 0}, EZ[3] = {1, 0, 0};
    const orc_grid *g = &w->g;
    const int r = w->r;
    const double dxx = axis_d2(f, g, w->lap, r, z, y, x, 0, 0, 1);
    const double dyy = axis_d2(f, g, w->lap, r, z, y, x, 0, 1, 0);
    const double dzz = axis_d2(f, g, w->lap, r, z, y, x, 1, 0, 0);
    const double dxy = mixed_d2(f, g, t->d1, r, z, y, x, EX, EY);
    const double dyz = mixed_d2(f, g, t->d1, r, z, y, x, EY, EZ);
    const double dxz = mixed_d2(f, g, t->d1, r, z, y, x, EX, EZ);
    const long i = at(g, z, y, x);
    const double th = t->theta[i], ph = t->phi[i];
    const double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    *lf = dxx + dyy + dzz;
    *h1f = st * st * cp * cp * dxx + st * st * sp * sp * dyy + ct * ct * dzz +
           st * st * sin(2.0 * ph) * dxy + sin(2.0 * th) * sp * dyz + sin(2.0 * th) * cp * dxz;
}

/* L f and H1 f on the interior of a padded field (zero elsewhere) */
void orc_tti_operators(const orc_wave *w, const orc_tti *t, const double *f, double *lf,
                       double *h1f) {
    const orc_grid *g = &w->g;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                const long i = at(g, z, y, x);
                tti_ops(w, t, f, z, y, x, &lf[i], &h1f[i]);
            }
}

static void tti_step_with_G(const orc_wave *w, const orc_tti *t, const double *G, int n,
                            const double *pp, const double *pc, double *pn, const double *qp,
                            const double *qc, double *qn, double *trace) {
    const orc_grid *g = &w->g;
    const double sg = t->sigma, al = t->alpha;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->nz; ++z)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) {
                double lp, h1p, lq, h1q;
                tti_ops(w, t, pc, z, y, x, &lp, &h1p);
                tti_ops(w, t, qc, z, y, x, &lq, &h1q);
                const double h2p = lp - h1p, h2q = lq - h1q;
                const long i = at(g, z, y, x);
                const double rp = (1.0 + 2.0 * t->eps[i]) * h2p + al * h1q + sg * (h1p - al * h1q);
                const double rq = (1.0 + 2.0 * t->delta[i]) / al * h2p + h1q - sg * (h2p / al - h2q);
                pn[i] = G[i] * (2.0 * pc[i] - G[i] * pp[i] + w->c2[i] * rp);
                qn[i] = G[i] * (2.0 * qc[i] - G[i] * qp[i] + w->c2[i] * rq);
            }
    if (n >= 0 && n < w->nt) {
        const long s = at(g, w->src_z, w->src_y, w->src_x);
        pn[s] += w->src[n];
        qn[s] += w->src[n];
    }
    if (trace)
        for (long y = 0; y < g->ny; ++y)
            for (long x = 0; x < g->nx; ++x) trace[y * g->nx + x] = pc[at(g, 0, y, x)];
}

void orc_tti_step(const orc_wave *w, const orc_tti *t, int n, const double *pp, const double *pc,
                  double *pn, const double *qp, const double *qc, double *qn, double *trace) {
    double *G = sponge_field(w);
    tti_step_with_G(w, t, G, n, pp, pc, pn, qp, qc, qn, trace);
    free(G);
}

/* Forward TTI run from (p^0, p^1, q^0, q^1); traces [nt][ny][nx] of p; last receives
 * p^{nt-1}, p^nt, q^{nt-1}, q^nt when non-NULL. */
void orc_tti_forward(const orc_wave *w, const orc_tti *t, const double *p0, const double *p1,
                     const double *q0, const double *q1, double *traces, double *last) {
    const orc_grid *g = &w->g;
    const size_t L = field_len(g);
    double *G = sponge_field(w);
    double *P[3], *Q[3];
    for (int i = 0; i < 3; ++i) {
        P[i] = calloc(L, sizeof(double));
        Q[i] = calloc(L, sizeof(double));
    }
    memcpy(P[0], p0, L * sizeof(double)); memcpy(P[1], p1, L * sizeof(double));
    memcpy(Q[0], q0, L * sizeof(double)); memcpy(Q[1], q1, L * sizeof(double));
    for (long y = 0; y < g->ny; ++y)
        for (long x = 0; x < g->nx; ++x) traces[y * g->nx + x] = p0[at(g, 0, y, x)];
    for (int n = 1; n < w->nt; ++n)
        tti_step_with_G(w, t, G, n, P[(n - 1) % 3], P[n % 3], P[(n + 1) % 3], Q[(n - 1) % 3],
                        Q[n % 3], Q[(n + 1) % 3], traces + (size_t)n * g->ny * g->nx);
    if (last) {
        const int m = w->nt;
        memcpy(last, P[(m - 1) % 3], L * sizeof(double));
        memcpy(last + L, P[m % 3], L * sizeof(double));
        memcpy(last + 2 * L, Q[(m - 1) % 3], L * sizeof(double));
        memcpy(last + 3 * L, Q[m % 3], L * sizeof(double));
    }
    for (int i = 0; i < 3; ++i) { free(P[i]); free(Q[i]); }
    free(G);
}
