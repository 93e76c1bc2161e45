/*
 * FP64 CPU oracle for the per-projection PCA solve -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no source with the HIP library: every
 * routine here is the plain definition from the paper (Li et al., "3D tumor
 * localization through real-time volumetric x-ray imaging for lung cancer
 * radiotherapy"), written for a reader to check by eye, in double precision,
 * built with -O2 -ffp-contract=off and no fast-math.
 *
 * Conventions (the paper's 1-based (i, j, k) of the Appendix become 0-based):
 *   volume  f[i + n1*(j + n2*k)], voxel centre = origin + (i, j, k) * spacing
 *   DVF     x[c*N + v], c = 0 lateral, 1 AP, 2 SI, in mm (pull-back field)
 *   modes   U[(k*3 + c)*N + v]
 *   image   p[iu + nu*iv]
 *
 * Readings of points the paper leaves open (the projection operator's
 * discretisation, zero extension outside the grid, ...) are documented with
 * each function.  OpenMP is used only for loops whose iterations are
 * independent, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n[3];
    double spacing[3];
    double origin[3];
} orc_vol;

typedef struct {
    double angle, sad, sid;
    int32_t nu, nv;
    double pitch_u, pitch_v, offset_u, offset_v, step;
} orc_proj;

typedef struct {
    double src[3];   /* source position (mm) */
    double dir[3];   /* unit direction */
    double t_in;     /* entry distance along dir (mm) */
    double length;   /* chord length through the box (mm), 0 if missed */
    int64_t nsamp;   /* ceil(length / step) */
    double dt;       /* length / nsamp */
} orc_ray;

/* ------------------------------------------------------------------------
 * Trilinear interpolation with zero extension (Appendix, Eq. A.5).
 * q is a position in voxel-index units; neighbours outside [0, n-1] read 0.
 * ---------------------------------------------------------------------- */
static double voxel_or_zero(const orc_vol *vol, const double *f, int64_t i, int64_t j, int64_t k)
{
    if (i < 0 || j < 0 || k < 0 || i >= vol->n[0] || j >= vol->n[1] || k >= vol->n[2])
        return 0.0;
    return f[i + (int64_t)vol->n[0] * (j + (int64_t)vol->n[1] * k)];
}

static double trilinear(const orc_vol *vol, const double *f, const double q[3])
{
    /* l, m, n: integer parts; z1, z2, z3: fractional parts (Eq. A.5) */
    double fl = floor(q[0]), fm = floor(q[1]), fn = floor(q[2]);
    int64_t l = (int64_t)fl, m = (int64_t)fm, n = (int64_t)fn;
    double z1 = q[0] - fl, z2 = q[1] - fm, z3 = q[2] - fn;
    return voxel_or_zero(vol, f, l,     m,     n)     * (1 - z1) * (1 - z2) * (1 - z3)
         + voxel_or_zero(vol, f, l + 1, m,     n)     * z1 * (1 - z2) * (1 - z3)
         + voxel_or_zero(vol, f, l,     m + 1, n)     * (1 - z1) * z2 * (1 - z3)
         + voxel_or_zero(vol, f, l,     m,     n + 1) * (1 - z1) * (1 - z2) * z3
         + voxel_or_zero(vol, f, l + 1, m + 1, n)     * z1 * z2 * (1 - z3)
         + voxel_or_zero(vol, f, l + 1, m,     n + 1) * z1 * (1 - z2) * z3
         + voxel_or_zero(vol, f, l,     m + 1, n + 1) * (1 - z1) * z2 * z3
         + voxel_or_zero(vol, f, l + 1, m + 1, n + 1) * z1 * z2 * z3;
}

/* ------------------------------------------------------------------------
 * Cone-beam geometry for one projection (Sec. II.A: P is "a projection
 * matrix which computes the projection image of f"; it changes with the
 * gantry angle).  Reading: circular orbit about the SI axis, source at
 * (SAD sin t, -SAD cos t, 0), flat detector SID from the source, one ray per
 * pixel centre, fixed-step midpoint rule over the chord through the box
 * spanned by the first and last voxel centres.
 * ---------------------------------------------------------------------- */
void orc_ray_setup(const orc_vol *vol, const orc_proj *pr, int32_t iu, int32_t iv, orc_ray *ray)
{
    double st = sin(pr->angle), ct = cos(pr->angle);
    double S[3] = { pr->sad * st, -pr->sad * ct, 0.0 };
    double mag = (pr->sid - pr->sad) / pr->sad;
    double D[3] = { -mag * S[0], -mag * S[1], 0.0 };
    double eu[3] = { ct, st, 0.0 };
    double ev[3] = { 0.0, 0.0, 1.0 };
    double u = (iu - 0.5 * (pr->nu - 1)) * pr->pitch_u + pr->offset_u;
    double v = (iv - 0.5 * (pr->nv - 1)) * pr->pitch_v + pr->offset_v;
    double d[3], len = 0.0;
    for (int c = 0; c < 3; ++c) {
        double P = D[c] + u * eu[c] + v * ev[c];
        d[c] = P - S[c];
        len += d[c] * d[c];
    }
    len = sqrt(len);
    for (int c = 0; c < 3; ++c) {
        ray->src[c] = S[c];
        ray->dir[c] = d[c] / len;
    }
    /* slab method against the box [origin, origin + (n-1) * spacing] */
    double t0 = -INFINITY, t1 = INFINITY;
    int missed = 0;
    for (int c = 0; c < 3; ++c) {
        double lo = vol->origin[c];
        double hi = vol->origin[c] + (vol->n[c] - 1) * vol->spacing[c];
        if (ray->dir[c] == 0.0) {
            if (S[c] < lo || S[c] > hi) missed = 1;
            continue;
        }
        double ta = (lo - S[c]) / ray->dir[c];
        double tb = (hi - S[c]) / ray->dir[c];
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    double L = t1 - t0;
    if (missed || !(L > 0.0)) {
        ray->t_in = 0.0; ray->length = 0.0; ray->nsamp = 0; ray->dt = 0.0;
        return;
    }
    ray->t_in = t0;
    ray->length = L;
    ray->nsamp = (int64_t)ceil(L / pr->step);
    ray->dt = L / (double)ray->nsamp;
}

static void sample_position(const orc_vol *vol, const orc_ray *ray, int64_t s, double q[3])
{
    double t = ray->t_in + ((double)s + 0.5) * ray->dt;
    for (int c = 0; c < 3; ++c) {
        double X = ray->src[c] + t * ray->dir[c];
        q[c] = (X - vol->origin[c]) / vol->spacing[c];
    }
}

/* One detector pixel of P f (Eq. 2): dt * sum_s f~(sample s). */
double orc_drr_pixel(const orc_vol *vol, const orc_proj *pr, const double *f, int32_t iu, int32_t iv)
{
    orc_ray ray;
    orc_ray_setup(vol, pr, iu, iv, &ray);
    double acc = 0.0;
    for (int64_t s = 0; s < ray.nsamp; ++s) {
        double q[3];
        sample_position(vol, &ray, s, q);
        acc += trilinear(vol, f, q);
    }
    return ray.dt * acc;
}

/* P f for the whole detector. */
void orc_drr_forward(const orc_vol *vol, const orc_proj *pr, const double *f, double *p)
{
    int64_t M = (int64_t)pr->nu * pr->nv;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < M; ++r)
        p[r] = orc_drr_pixel(vol, pr, f, (int32_t)(r % pr->nu), (int32_t)(r / pr->nu));
}

/* Selected pixels of P f (full-size parity on a sample of rays). */
void orc_drr_pixels(const orc_vol *vol, const orc_proj *pr, const double *f,
                    int64_t count, const int64_t *pix, double *p)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t)
        p[t] = orc_drr_pixel(vol, pr, f, (int32_t)(pix[t] % pr->nu), (int32_t)(pix[t] / pr->nu));
}

/* Scatter of the rays of detector rows [iv0, iv1) into bp (not cleared):
 * every sample sends dt * r to the same eight voxels, with the same
 * trilinear weights, that orc_drr_pixel reads it from. */
static void adjoint_rows(const orc_vol *vol, const orc_proj *pr, const double *r, int32_t iv0,
                         int32_t iv1, double *bp)
{
    for (int32_t iv = iv0; iv < iv1; ++iv)
        for (int32_t iu = 0; iu < pr->nu; ++iu) {
            double rr = r[iu + (int64_t)pr->nu * iv];
            orc_ray ray;
            orc_ray_setup(vol, pr, iu, iv, &ray);
            if (ray.nsamp == 0 || rr == 0.0) continue;
            double c = ray.dt * rr;
            for (int64_t s = 0; s < ray.nsamp; ++s) {
                double q[3];
                sample_position(vol, &ray, s, q);
                double fl[3], z[3];
                int64_t b[3];
                for (int a = 0; a < 3; ++a) {
                    fl[a] = floor(q[a]);
                    b[a] = (int64_t)fl[a];
                    z[a] = q[a] - fl[a];
                }
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di) {
                            int64_t i = b[0] + di, j = b[1] + dj, k = b[2] + dk;
                            if (i < 0 || j < 0 || k < 0 || i >= vol->n[0] || j >= vol->n[1] || k >= vol->n[2])
                                continue;
                            double wgt = (di ? z[0] : 1 - z[0]) * (dj ? z[1] : 1 - z[1]) * (dk ? z[2] : 1 - z[2]);
                            bp[i + (int64_t)vol->n[0] * (j + (int64_t)vol->n[1] * k)] += c * wgt;
                        }
            }
        }
}

/* P^T r (the back-projection in the gradient of the Appendix): the literal
 * transpose of orc_drr_forward.  The detector rows are cut into a fixed
 * number of bands (up to 16, fewer when the private copies would pass
 * 2 GiB); each band scatters into a private zeroed volume (bands run in
 * parallel), then every voxel sums the bands in band order.  The partition
 * and the order depend only on the sizes, never on the thread count, so the
 * result is the same bits on any machine. */
void orc_drr_adjoint(const orc_vol *vol, const orc_proj *pr, const double *r, double *bp)
{
    int64_t N = (int64_t)vol->n[0] * vol->n[1] * vol->n[2];
    int64_t cap = ((int64_t)1 << 31) / (N * (int64_t)sizeof(double));
    int32_t nb = cap < 1 ? 1 : (cap > 16 ? 16 : (int32_t)cap);
    if (nb > pr->nv) nb = pr->nv;
    if (nb <= 1) {
        memset(bp, 0, (size_t)N * sizeof(double));
        adjoint_rows(vol, pr, r, 0, pr->nv, bp);
        return;
    }
    double *part = (double *)calloc((size_t)nb * (size_t)N, sizeof(double));
    if (!part) {   /* no room for the private copies: one sequential band */
        memset(bp, 0, (size_t)N * sizeof(double));
        adjoint_rows(vol, pr, r, 0, pr->nv, bp);
        return;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < nb; ++t) {
        int32_t iv0 = (int32_t)((int64_t)pr->nv * t / nb);
        int32_t iv1 = (int32_t)((int64_t)pr->nv * (t + 1) / nb);
        adjoint_rows(vol, pr, r, iv0, iv1, part + (int64_t)t * N);
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < N; ++v) {
        double acc = 0.0;
        for (int32_t t = 0; t < nb; ++t)
            acc += part[(int64_t)t * N + v];
        bp[v] = acc;
    }
    free(part);
}

/* Eq. 1: x = xbar + sum_k u_k w_k.  mean may be NULL (zero mean). */
void orc_pca_dvf(int64_t N, int32_t K, const double *mean, const double *U, const double *w, double *x)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < 3 * N; ++e) {
        double acc = mean ? mean[e] : 0.0;
        for (int32_t k = 0; k < K; ++k)
            acc += U[(int64_t)k * 3 * N + e] * w[k];
        x[e] = acc;
    }
}

/* Eq. A.3 with Eq. A.5: f(i,j,k) = f0(i + x1/s1, j + x2/s2, k + x3/s3); the
 * DVF is given in mm and divided by the spacing to reach index units. */
void orc_warp(const orc_vol *vol, const double *f0, const double *x, double *f)
{
    int64_t n1 = vol->n[0], n2 = vol->n[1], n3 = vol->n[2], N = n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n3; ++k)
        for (int64_t j = 0; j < n2; ++j)
            for (int64_t i = 0; i < n1; ++i) {
                int64_t v = i + n1 * (j + n2 * k);
                double q[3] = { i + x[v] / vol->spacing[0],
                                j + x[N + v] / vol->spacing[1],
                                k + x[2 * N + v] / vol->spacing[2] };
                f[v] = trilinear(vol, f0, q);
            }
}

/* Eq. A.8 and its two analogues: the diagonal Jacobian df/dx_c at every
 * voxel, per mm (the index-unit derivative divided by the spacing).  At an
 * integer position the floor convention gives the right-side derivative. */
void orc_warp_jacobian(const orc_vol *vol, const double *f0, const double *x, double *jac)
{
    int64_t n1 = vol->n[0], n2 = vol->n[1], n3 = vol->n[2], N = n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n3; ++k)
        for (int64_t j = 0; j < n2; ++j)
            for (int64_t i = 0; i < n1; ++i) {
                int64_t v = i + n1 * (j + n2 * k);
                double q1 = i + x[v] / vol->spacing[0];
                double q2 = j + x[N + v] / vol->spacing[1];
                double q3 = k + x[2 * N + v] / vol->spacing[2];
                double fl1 = floor(q1), fl2 = floor(q2), fl3 = floor(q3);
                int64_t l = (int64_t)fl1, m = (int64_t)fl2, n = (int64_t)fl3;
                double z1 = q1 - fl1, z2 = q2 - fl2, z3 = q3 - fl3;
#define F0(a, b, c) voxel_or_zero(vol, f0, (a), (b), (c))
                double d1 = (F0(l + 1, m, n) - F0(l, m, n)) * (1 - z2) * (1 - z3)
                          + (F0(l + 1, m + 1, n) - F0(l, m + 1, n)) * z2 * (1 - z3)
                          + (F0(l + 1, m, n + 1) - F0(l, m, n + 1)) * (1 - z2) * z3
                          + (F0(l + 1, m + 1, n + 1) - F0(l, m + 1, n + 1)) * z2 * z3;
                double d2 = (F0(l, m + 1, n) - F0(l, m, n)) * (1 - z1) * (1 - z3)
                          + (F0(l + 1, m + 1, n) - F0(l + 1, m, n)) * z1 * (1 - z3)
                          + (F0(l, m + 1, n + 1) - F0(l, m, n + 1)) * (1 - z1) * z3
                          + (F0(l + 1, m + 1, n + 1) - F0(l + 1, m, n + 1)) * z1 * z3;
                double d3 = (F0(l, m, n + 1) - F0(l, m, n)) * (1 - z1) * (1 - z2)
                          + (F0(l + 1, m, n + 1) - F0(l + 1, m, n)) * z1 * (1 - z2)
                          + (F0(l, m + 1, n + 1) - F0(l, m + 1, n)) * (1 - z1) * z2
                          + (F0(l + 1, m + 1, n + 1) - F0(l + 1, m + 1, n)) * z1 * z2;
#undef F0
                jac[v] = d1 / vol->spacing[0];
                jac[N + v] = d2 / vol->spacing[1];
                jac[2 * N + v] = d3 / vol->spacing[2];
            }
}

/* Gradient chain of the Appendix: dJ/dw = 2 U^T (df/dx) P^T r, with the
 * diagonal Jacobian applied component-wise.  The voxels are cut into 64
 * fixed chunks summed in parallel; the chunk sums are added in chunk order,
 * so the result does not depend on the thread count. */
void orc_grad_chain(int64_t N, int32_t K, const double *U, const double *jac, const double *bp, double *g)
{
    enum { NCH = 64 };
    double *part = (double *)malloc((size_t)NCH * (size_t)K * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < NCH; ++t) {
        int64_t v0 = N * t / NCH, v1 = N * (t + 1) / NCH;
        for (int32_t k = 0; k < K; ++k) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double *u = U + ((int64_t)k * 3 + c) * N;
                const double *jc = jac + (int64_t)c * N;
                for (int64_t v = v0; v < v1; ++v)
                    acc += u[v] * jc[v] * bp[v];
            }
            part[(int64_t)t * K + k] = acc;
        }
    }
    for (int32_t k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int t = 0; t < NCH; ++t)
            acc += part[(int64_t)t * K + k];
        g[k] = 2.0 * acc;
    }
    free(part);
}

/* Trilinear value of the DVF (Eq. 1 evaluated at the eight neighbours) at a
 * point y in mm; zero extension outside the grid. */
static void dvf_at_point(const orc_vol *vol, int32_t K, const double *mean, const double *U,
                         const double *w, const double y[3], double out[3])
{
    int64_t N = (int64_t)vol->n[0] * vol->n[1] * vol->n[2];
    double q[3], fl[3], z[3];
    int64_t b[3];
    for (int a = 0; a < 3; ++a) {
        q[a] = (y[a] - vol->origin[a]) / vol->spacing[a];
        fl[a] = floor(q[a]);
        b[a] = (int64_t)fl[a];
        z[a] = q[a] - fl[a];
    }
    out[0] = out[1] = out[2] = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                int64_t i = b[0] + di, j = b[1] + dj, k = b[2] + dk;
                if (i < 0 || j < 0 || k < 0 || i >= vol->n[0] || j >= vol->n[1] || k >= vol->n[2])
                    continue;
                int64_t v = i + (int64_t)vol->n[0] * (j + (int64_t)vol->n[1] * k);
                double wgt = (di ? z[0] : 1 - z[0]) * (dj ? z[1] : 1 - z[1]) * (dk ? z[2] : 1 - z[2]);
                for (int c = 0; c < 3; ++c) {
                    double xc = mean ? mean[(int64_t)c * N + v] : 0.0;
                    for (int32_t kk = 0; kk < K; ++kk)
                        xc += U[((int64_t)kk * 3 + c) * N + v] * w[kk];
                    out[c] += wgt * xc;
                }
            }
}

/* Tumour position (Sec. II.A, last paragraphs): the solved field is a
 * pull-back field, so the tumour centre c0 of the reference image moves to
 * the point y with y + x(y) = c0.  Fixed-point iteration y <- c0 - x(y) from
 * y = c0 (the inversion scheme the paper adopts from its ref. 18), applied at
 * this one point only.  Returns the iteration count, or -1 if not converged. */
int32_t orc_locate(const orc_vol *vol, int32_t K, const double *mean, const double *U,
                   const double *w, const double c0[3], double tol, int32_t max_iter, double out[3])
{
    double y[3] = { c0[0], c0[1], c0[2] };
    for (int32_t it = 1; it <= max_iter; ++it) {
        double x[3], yn[3], d2 = 0.0;
        dvf_at_point(vol, K, mean, U, w, y, x);
        for (int c = 0; c < 3; ++c) {
            yn[c] = c0[c] - x[c];
            d2 += (yn[c] - y[c]) * (yn[c] - y[c]);
            y[c] = yn[c];
        }
        if (sqrt(d2) < tol) {
            out[0] = y[0]; out[1] = y[1]; out[2] = y[2];
            return it;
        }
    }
    out[0] = y[0]; out[1] = y[1]; out[2] = y[2];
    return -1;
}

/* ------------------------------------------------------------------------
 * Exact radiological path (Siddon's method; the paper simulates its digital
 * projections with it, Sec. II.B).  The volume is read as piecewise constant
 * over voxel cells [centre - s/2, centre + s/2]; a ray's value is the sum
 * over cells of (length of the ray inside the cell) * (cell value).  Written
 * in the original formulation: every crossing parameter of the ray with a
 * cell plane inside the grid's outer box is collected and sorted; each
 * interval between consecutive crossings lies in one cell, found from its
 * midpoint.  The ray runs from the source to the pixel centre.
 * ---------------------------------------------------------------------- */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

double orc_siddon_pixel(const orc_vol *vol, const orc_proj *pr, const double *f, int32_t iu,
                        int32_t iv)
{
    double st = sin(pr->angle), ct = cos(pr->angle);
    double S[3] = { pr->sad * st, -pr->sad * ct, 0.0 };
    double mag = (pr->sid - pr->sad) / pr->sad;
    double Dc[3] = { -mag * S[0], -mag * S[1], 0.0 };
    double eu[3] = { ct, st, 0.0 };
    double ev[3] = { 0.0, 0.0, 1.0 };
    double u = (iu - 0.5 * (pr->nu - 1)) * pr->pitch_u + pr->offset_u;
    double v = (iv - 0.5 * (pr->nv - 1)) * pr->pitch_v + pr->offset_v;
    double d[3], len2 = 0.0, b0[3], bn[3];
    for (int c = 0; c < 3; ++c) {
        d[c] = Dc[c] + u * eu[c] + v * ev[c] - S[c];   /* source -> pixel, alpha in [0, 1] */
        len2 += d[c] * d[c];
        b0[c] = vol->origin[c] - 0.5 * vol->spacing[c];
        bn[c] = vol->origin[c] + (vol->n[c] - 0.5) * vol->spacing[c];
    }
    double amin = 0.0, amax = 1.0;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) {
            if (S[c] <= b0[c] || S[c] >= bn[c]) return 0.0;
            continue;
        }
        double a0 = (b0[c] - S[c]) / d[c], a1 = (bn[c] - S[c]) / d[c];
        if (a0 > a1) { double t = a0; a0 = a1; a1 = t; }
        if (a0 > amin) amin = a0;
        if (a1 < amax) amax = a1;
    }
    if (!(amin < amax)) return 0.0;
    int64_t cap = 2 + (int64_t)vol->n[0] + vol->n[1] + vol->n[2] + 3;
    double *al = (double *)malloc((size_t)cap * sizeof(double));
    int64_t m = 0;
    al[m++] = amin;
    al[m++] = amax;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) continue;
        for (int32_t i = 0; i <= vol->n[c]; ++i) {
            double a = (b0[c] + i * vol->spacing[c] - S[c]) / d[c];
            if (a > amin && a < amax) al[m++] = a;
        }
    }
    qsort(al, (size_t)m, sizeof(double), cmp_double);
    double sum = 0.0, L = sqrt(len2);
    for (int64_t k = 0; k + 1 < m; ++k) {
        double da = al[k + 1] - al[k];
        if (!(da > 0.0)) continue;
        double mid = 0.5 * (al[k] + al[k + 1]);
        int64_t idx[3];
        for (int c = 0; c < 3; ++c) {
            double X = S[c] + mid * d[c];
            int64_t i = (int64_t)floor((X - b0[c]) / vol->spacing[c]);
            if (i < 0) i = 0;
            if (i > vol->n[c] - 1) i = vol->n[c] - 1;
            idx[c] = i;
        }
        sum += da * L * f[idx[0] + (int64_t)vol->n[0] * (idx[1] + (int64_t)vol->n[1] * idx[2])];
    }
    free(al);
    return sum;
}

void orc_siddon_forward(const orc_vol *vol, const orc_proj *pr, const double *f, double *p)
{
    int64_t M = (int64_t)pr->nu * pr->nv;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < M; ++r)
        p[r] = orc_siddon_pixel(vol, pr, f, (int32_t)(r % pr->nu), (int32_t)(r / pr->nu));
}

/* Ray records for a whole detector (used by tests for chord pins). */
void orc_ray_table(const orc_vol *vol, const orc_proj *pr, double *t_in, double *length,
                   int64_t *nsamp, double *dt)
{
    int64_t M = (int64_t)pr->nu * pr->nv;
    for (int64_t r = 0; r < M; ++r) {
        orc_ray ray;
        orc_ray_setup(vol, pr, (int32_t)(r % pr->nu), (int32_t)(r / pr->nu), &ray);
        t_in[r] = ray.t_in;
        length[r] = ray.length;
        nsamp[r] = ray.nsamp;
        dt[r] = ray.dt;
    }
}

/* Thread count of the parallel loops (the CPU baseline times 1 and all cores);
 * results do not depend on it.  Returns the count now in force. */
int32_t orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
