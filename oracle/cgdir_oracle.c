/*
 * FP64 CPU oracle for contour-guided demons registration (CG-DIR).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the CPU
 * baseline of the benchmark, never by the registration library.  Written from the
 * paper (section 2.1, Eqs. 1-7; section 2.2 and Algorithm A) as plain loops in double
 * precision.  The voxel loops are OpenMP-parallel over independent voxels only; no
 * step is blocked, fused or reordered.
 *
 * Readings of the paper taken here (the HIP library takes the same ones):
 *  - modified images use CT numbers, I_i = (1 + s_i M_i / 2)(I_0 + c0), c0 = 1000 HU;
 *  - the gradient is central differences of the warped image, indices clamped;
 *  - interpolation is trilinear with the sample position clamped to the volume;
 *  - warping pulls back on the target grid: (I o u)(x) = I(x + u(x));
 *  - |grad I0~| = 0 gives du = 0;  beta = (T0 - I0~)^2 exactly;
 *  - Gaussian: sampled, radius ceil(3 sigma), normalised, clamped, x then y then z;
 *  - composite update u <- du + u o (Id + du);
 *  - restriction keeps the even voxels of the sigma=1 smoothed image, dims ceil(n/2);
 *    prolongation is 2 u(x/2);
 *  - UROI: union of the target structures dilated by an ellipsoid (5, 5, 4) voxels;
 *  - stopping: after every `window` finest-level iterations, stop when
 *    delta_{n-window} - delta_n <= eps (n = the last iteration run).
 *
 * Parity unpinned: no number in the paper tests these readings, so the pins check each
 * function against its definition and library routines but not the choice itself: c0, the
 * restriction's sigma = 1 filter, the UROI's ellipsoid, the form of the stopping rule, the
 * clamped borders of the gradient, the interpolation and the Gaussian, the per-level voxel
 * size spacing * 2^l, and the coarse-level masks taken at the voxels the restriction keeps.
 */
#include "cgdir_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, l) ((size_t)(i) + (size_t)nx * ((size_t)(j) + (size_t)ny * (size_t)(l)))

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int bad_dims(int nx, int ny, int nz) { return nx < 1 || ny < 1 || nz < 1; }

/* ---------------------------------------------------------------- Gaussian (section 2.2) */

int orc_gauss_radius(double sigma)
{
    if (!(sigma > 0.0)) return 0;
    return (int)ceil(3.0 * sigma);
}

int orc_gauss_weights(double sigma, double *w)
{
    int R = orc_gauss_radius(sigma);
    if (R == 0) {
        w[0] = 1.0;
        return 0;
    }
    double sum = 0.0;
    for (int m = -R; m <= R; ++m) {
        w[m + R] = exp(-(double)(m * m) / (2.0 * sigma * sigma));
        sum += w[m + R];
    }
    for (int m = 0; m < 2 * R + 1; ++m) w[m] /= sum;
    return R;
}

/* one 1D pass along axis `ax` (0 = x, 1 = y, 2 = z) with clamped indices */
static void smooth_axis(const double *f, int nx, int ny, int nz, int ax, const double *w, int R,
                        double *out)
{
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int m = -R; m <= R; ++m) {
                    int ii = i, jj = j, ll = l;
                    if (ax == 0) ii = clampi(i + m, 0, nx - 1);
                    if (ax == 1) jj = clampi(j + m, 0, ny - 1);
                    if (ax == 2) ll = clampi(l + m, 0, nz - 1);
                    s += w[m + R] * f[IDX(ii, jj, ll)];
                }
                out[IDX(i, j, l)] = s;
            }
}

int orc_smooth_axes(const double *f, int nx, int ny, int nz, const double sigma[3], double *out)
{
    if (bad_dims(nx, ny, nz) || f == out) return -1;
    size_t n = (size_t)nx * ny * nz;
    double *a = (double *)malloc(sizeof(double) * n);
    double *b = (double *)malloc(sizeof(double) * n);
    const double *src[3] = {f, a, b};
    double *dst[3] = {a, b, out};
    for (int ax = 0; ax < 3; ++ax) {
        int R = orc_gauss_radius(sigma[ax]);
        double *w = (double *)malloc(sizeof(double) * (size_t)(2 * R + 1));
        orc_gauss_weights(sigma[ax], w);
        smooth_axis(src[ax], nx, ny, nz, ax, w, R, dst[ax]);
        free(w);
    }
    free(a);
    free(b);
    return 0;
}

int orc_smooth(const double *f, int nx, int ny, int nz, double sigma, double *out)
{
    const double s[3] = {sigma, sigma, sigma};
    return orc_smooth_axes(f, nx, ny, nz, s, out);
}

/* ---------------------------------------------------------------- interpolation (kernel 4) */

/* position clamped to [0, n-1]; i0 = floor, i1 = min(i0 + 1, n - 1), t = p - i0 */
static void axis_split(double p, int n, int *i0, int *i1, double *t)
{
    double pc = p < 0.0 ? 0.0 : (p > (double)(n - 1) ? (double)(n - 1) : p);
    int a = (int)floor(pc);
    if (a > n - 1) a = n - 1;
    *i0 = a;
    *i1 = a + 1 <= n - 1 ? a + 1 : n - 1;
    *t = pc - (double)a;
}

static double lerp(double a, double b, double t) { return a + t * (b - a); }

double orc_sample(const double *f, int nx, int ny, int nz, double px, double py, double pz)
{
    int x0, x1, y0, y1, z0, z1;
    double tx, ty, tz;
    axis_split(px, nx, &x0, &x1, &tx);
    axis_split(py, ny, &y0, &y1, &ty);
    axis_split(pz, nz, &z0, &z1, &tz);
    double c00 = lerp(f[IDX(x0, y0, z0)], f[IDX(x1, y0, z0)], tx);
    double c10 = lerp(f[IDX(x0, y1, z0)], f[IDX(x1, y1, z0)], tx);
    double c01 = lerp(f[IDX(x0, y0, z1)], f[IDX(x1, y0, z1)], tx);
    double c11 = lerp(f[IDX(x0, y1, z1)], f[IDX(x1, y1, z1)], tx);
    double c0 = lerp(c00, c10, ty);
    double c1 = lerp(c01, c11, ty);
    return lerp(c0, c1, tz);
}

int orc_warp(const double *f, int nx, int ny, int nz, const double *u, double *out)
{
    if (bad_dims(nx, ny, nz)) return -1;
    size_t n = (size_t)nx * ny * nz;
    const double *ux = u, *uy = u + n, *uz = u + 2 * n;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t v = IDX(i, j, l);
                out[v] = orc_sample(f, nx, ny, nz, i + ux[v], j + uy[v], l + uz[v]);
            }
    return 0;
}

int orc_warp_mask(const uint8_t *m, int nx, int ny, int nz, const double *u, uint8_t *out)
{
    if (bad_dims(nx, ny, nz)) return -1;
    size_t n = (size_t)nx * ny * nz;
    double *f = (double *)calloc(n, sizeof(double));
    double *w = (double *)calloc(n, sizeof(double));
    for (size_t v = 0; v < n; ++v) f[v] = m[v] ? 1.0 : 0.0;
    orc_warp(f, nx, ny, nz, u, w);
    for (size_t v = 0; v < n; ++v) out[v] = w[v] >= 0.5 ? 1 : 0;
    free(f);
    free(w);
    return 0;
}

/* ---------------------------------------------------------------- Eq.7 (kernel 3) */

/* v minimising E1(v) of Eq.6 with beta = d^2 (Thirion):
 *   v = (a0 d + sum_i lambda_i a_i d_i) / (a0^2 + sum_i lambda_i a_i^2 + d^2)        */
double orc_eq7(double a0, double d, int k, const double *lambda, const double *a, const double *di)
{
    double num = a0 * d;
    double den = a0 * a0 + d * d;
    for (int i = 0; i < k; ++i) {
        num += lambda[i] * a[i] * di[i];
        den += lambda[i] * a[i] * a[i];
    }
    return num / den;
}

/* ---------------------------------------------------------------- gradient (kernel 2) */

/* central differences divided by twice the voxel size h of each axis */
static void grad_at(const double *f, int nx, int ny, int nz, int i, int j, int l, const double h[3], double g[3])
{
    g[0] = (f[IDX(clampi(i + 1, 0, nx - 1), j, l)] - f[IDX(clampi(i - 1, 0, nx - 1), j, l)]) / (2.0 * h[0]);
    g[1] = (f[IDX(i, clampi(j + 1, 0, ny - 1), l)] - f[IDX(i, clampi(j - 1, 0, ny - 1), l)]) / (2.0 * h[1]);
    g[2] = (f[IDX(i, j, clampi(l + 1, 0, nz - 1))] - f[IDX(i, j, clampi(l - 1, 0, nz - 1))]) / (2.0 * h[2]);
}

static const double kUnit[3] = {1.0, 1.0, 1.0};

int orc_gradient(const double *f, int nx, int ny, int nz, double *g)
{
    return orc_gradient_h(f, nx, ny, nz, NULL, g);
}

int orc_gradient_h(const double *f, int nx, int ny, int nz, const double *h, double *g)
{
    if (bad_dims(nx, ny, nz)) return -1;
    if (!h) h = kUnit;
    size_t n = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double gv[3];
                grad_at(f, nx, ny, nz, i, j, l, h, gv);
                size_t v = IDX(i, j, l);
                g[v] = gv[0];
                g[n + v] = gv[1];
                g[2 * n + v] = gv[2];
            }
    return 0;
}

int orc_force(const double *wI0, const double *T0, int k, const double *const *wIp,
              const double *const *Tp, const double *lambda, int nx, int ny, int nz,
              double *du)
{
    return orc_force_h(wI0, T0, k, wIp, Tp, lambda, nx, ny, nz, NULL, du);
}

int orc_force_h(const double *wI0, const double *T0, int k, const double *const *wIp,
                const double *const *Tp, const double *lambda, int nx, int ny, int nz,
                const double *h, double *du)
{
    if (bad_dims(nx, ny, nz) || k < 0 || k > ORC_MAX_STRUCTS) return -1;
    if (!h) h = kUnit;
    size_t n = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t v = IDX(i, j, l);
                double g0[3];
                grad_at(wI0, nx, ny, nz, i, j, l, h, g0);
                double a02 = g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2];
                if (a02 == 0.0) { /* the direction n is undefined: no displacement */
                    du[v] = du[n + v] = du[2 * n + v] = 0.0;
                    continue;
                }
                double a0 = sqrt(a02);
                double nv[3] = {g0[0] / a0, g0[1] / a0, g0[2] / a0};
                double d = T0[v] - wI0[v];
                double a[ORC_MAX_STRUCTS], di[ORC_MAX_STRUCTS];
                for (int s = 0; s < k; ++s) {
                    double gi[3];
                    grad_at(wIp[s], nx, ny, nz, i, j, l, h, gi);
                    a[s] = gi[0] * nv[0] + gi[1] * nv[1] + gi[2] * nv[2];
                    di[s] = Tp[s][v] - wIp[s][v];
                }
                /* v n is the step in the length unit of h; the field is kept in voxels */
                double vv = orc_eq7(a0, d, k, lambda, a, di);
                du[v] = vv * nv[0] / h[0];
                du[n + v] = vv * nv[1] / h[1];
                du[2 * n + v] = vv * nv[2] / h[2];
            }
    return 0;
}

/* ---------------------------------------------------------------- composite update */

int orc_compose(const double *u, const double *du, int nx, int ny, int nz, double *uc)
{
    if (bad_dims(nx, ny, nz)) return -1;
    size_t n = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t v = IDX(i, j, l);
                double px = i + du[v], py = j + du[n + v], pz = l + du[2 * n + v];
                for (int c = 0; c < 3; ++c)
                    uc[c * n + v] = du[c * n + v] + orc_sample(u + c * n, nx, ny, nz, px, py, pz);
            }
    return 0;
}

/* ---------------------------------------------------------------- pyramid */

int orc_restrict(const double *f, int nx, int ny, int nz, double sigma, double *out)
{
    if (bad_dims(nx, ny, nz)) return -1;
    size_t n = (size_t)nx * ny * nz;
    double *s = (double *)malloc(sizeof(double) * n);
    orc_smooth(f, nx, ny, nz, sigma, s);
    int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
    for (int l = 0; l < cz; ++l)
        for (int j = 0; j < cy; ++j)
            for (int i = 0; i < cx; ++i)
                out[(size_t)i + (size_t)cx * ((size_t)j + (size_t)cy * l)] = s[IDX(2 * i, 2 * j, 2 * l)];
    free(s);
    return 0;
}

int orc_decimate_masks(const uint8_t *m, int k, int nx, int ny, int nz, uint8_t *out)
{
    if (bad_dims(nx, ny, nz) || k < 0) return -1;
    size_t n = (size_t)nx * ny * nz;
    int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
    size_t cn = (size_t)cx * cy * cz;
    for (int s = 0; s < k; ++s)
        for (int l = 0; l < cz; ++l)
            for (int j = 0; j < cy; ++j)
                for (int i = 0; i < cx; ++i)
                    out[s * cn + (size_t)i + (size_t)cx * ((size_t)j + (size_t)cy * l)] =
                        m[s * n + IDX(2 * i, 2 * j, 2 * l)] != 0;
    return 0;
}

int orc_prolong(const double *uc, int cnx, int cny, int cnz, int fnx, int fny, int fnz, double *uf)
{
    if (bad_dims(cnx, cny, cnz) || bad_dims(fnx, fny, fnz)) return -1;
    if (cnx != (fnx + 1) / 2 || cny != (fny + 1) / 2 || cnz != (fnz + 1) / 2) return -1;
    size_t cn = (size_t)cnx * cny * cnz, fn = (size_t)fnx * fny * fnz;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < fnz; ++l)
        for (int j = 0; j < fny; ++j)
            for (int i = 0; i < fnx; ++i) {
                size_t v = (size_t)i + (size_t)fnx * ((size_t)j + (size_t)fny * l);
                for (int c = 0; c < 3; ++c)
                    uf[c * fn + v] = 2.0 * orc_sample(uc + c * cn, cnx, cny, cnz, 0.5 * i, 0.5 * j, 0.5 * l);
            }
    return 0;
}

/* ---------------------------------------------------------------- UROI (section 2.2) */

static void paint_dilated(const uint8_t *src, int nx, int ny, int nz, const int r[3], uint8_t *out)
{
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (!src[IDX(i, j, l)]) continue;
                for (int c = -r[2]; c <= r[2]; ++c)
                    for (int b = -r[1]; b <= r[1]; ++b)
                        for (int a = -r[0]; a <= r[0]; ++a) {
                            double q = 0.0;
                            if (r[0] > 0) q += (double)(a * a) / (double)(r[0] * r[0]);
                            if (r[1] > 0) q += (double)(b * b) / (double)(r[1] * r[1]);
                            if (r[2] > 0) q += (double)(c * c) / (double)(r[2] * r[2]);
                            if (q > 1.0) continue;
                            int ii = i + a, jj = j + b, ll = l + c;
                            if (ii < 0 || jj < 0 || ll < 0 || ii >= nx || jj >= ny || ll >= nz) continue;
                            out[IDX(ii, jj, ll)] = 1;
                        }
            }
}

int orc_uroi(const uint8_t *masks, int k, int nx, int ny, int nz, const int r[3], uint8_t *out)
{
    if (bad_dims(nx, ny, nz) || k < 0 || r[0] < 0 || r[1] < 0 || r[2] < 0) return -1;
    size_t n = (size_t)nx * ny * nz;
    uint8_t *uni = (uint8_t *)calloc(n, 1);
    for (int s = 0; s < k; ++s)
        for (size_t v = 0; v < n; ++v)
            if (masks[(size_t)s * n + v]) uni[v] = 1;
    memset(out, 0, n);
    paint_dilated(uni, nx, ny, nz, r, out);
    free(uni);
    return 0;
}

int orc_auto_sign(const double *T0, const uint8_t *mask, int nx, int ny, int nz, const int r[3])
{
    size_t n = (size_t)nx * ny * nz;
    uint8_t *m = (uint8_t *)calloc(n, 1);
    uint8_t *dil = (uint8_t *)calloc(n, 1);
    for (size_t v = 0; v < n; ++v) m[v] = mask[v] ? 1 : 0;
    paint_dilated(m, nx, ny, nz, r, dil);
    double si = 0.0, so = 0.0;
    size_t ni = 0, no = 0;
    for (size_t v = 0; v < n; ++v) {
        if (m[v]) { si += T0[v]; ++ni; }
        else if (dil[v]) { so += T0[v]; ++no; }
    }
    free(m);
    free(dil);
    if (ni == 0 || no == 0) return 1;
    return si / (double)ni >= so / (double)no ? 1 : -1;
}

/* ---------------------------------------------------------------- modified images (section 2.1) */

int orc_modified_image(const double *F, const uint8_t *mask, int s, double c0, size_t n, double *out)
{
    if (s != 1 && s != -1) return -1;
    for (size_t v = 0; v < n; ++v) {
        double M = mask[v] ? (double)s : 0.0;
        out[v] = (1.0 + 0.5 * M) * (F[v] + c0);
    }
    return 0;
}

/* ---------------------------------------------------------------- one iteration (Algorithm A) */

int orc_step(const double *I0, const double *T0, int nx, int ny, int nz, int k,
             const double *const *Iplus, const double *const *Tplus, const double *lambda,
             double sigma_f, double sigma_d, const double *h, const uint8_t *uroi, double norm_range,
             double *u, double *delta)
{
    if (bad_dims(nx, ny, nz) || k < 0 || k > ORC_MAX_STRUCTS) return -1;
    if (!h) h = kUnit;
    /* the Gaussians are given in the length unit of h: sigma / h voxels along each axis */
    const double sf[3] = {sigma_f / h[0], sigma_f / h[1], sigma_f / h[2]};
    const double sd[3] = {sigma_d / h[0], sigma_d / h[1], sigma_d / h[2]};
    size_t n = (size_t)nx * ny * nz;
    double *wI0 = (double *)malloc(sizeof(double) * n);
    double **wIp = (double **)malloc(sizeof(double *) * (size_t)(k > 0 ? k : 1));
    double *du = (double *)malloc(sizeof(double) * 3 * n);
    double *dus = (double *)malloc(sizeof(double) * 3 * n);
    double *uc = (double *)malloc(sizeof(double) * 3 * n);

    /* warp the moving image and the modified images with the current u */
    orc_warp(I0, nx, ny, nz, u, wI0);
    for (int s = 0; s < k; ++s) {
        wIp[s] = (double *)malloc(sizeof(double) * n);
        orc_warp(Iplus[s], nx, ny, nz, u, wIp[s]);
    }
    /* stopping metric from the intensity difference at the current u */
    if (delta) {
        double sum = 0.0;
        size_t cnt = 0;
        for (size_t v = 0; v < n; ++v)
            if (!uroi || uroi[v]) {
                double d = (T0[v] - wI0[v]) / norm_range;
                sum += d * d;
                ++cnt;
            }
        *delta = cnt ? sqrt(sum / (double)cnt) : 0.0;
    }
    /* step 1: gradients and Eq.7 */
    orc_force_h(wI0, T0, k, (const double *const *)wIp, Tplus, lambda, nx, ny, nz, h, du);
    /* step 2: smooth the displacement */
    for (int c = 0; c < 3; ++c) orc_smooth_axes(du + c * n, nx, ny, nz, sf, dus + c * n);
    /* step 3: composite update */
    orc_compose(u, dus, nx, ny, nz, uc);
    /* step 4: smooth the field */
    for (int c = 0; c < 3; ++c) orc_smooth_axes(uc + c * n, nx, ny, nz, sd, u + c * n);

    for (int s = 0; s < k; ++s) free(wIp[s]);
    free(wIp);
    free(wI0);
    free(du);
    free(dus);
    free(uc);
    return 0;
}

/* ---------------------------------------------------------------- Algorithm A */

int orc_register(const double *target, const double *moving, int nx, int ny, int nz, int k,
                 const uint8_t *tmasks, const uint8_t *mmasks, const orc_params *p,
                 const double *initial_u, double *u_out, double *delta_hist, int *iters_done)
{
    if (bad_dims(nx, ny, nz) || !p || k < 0 || k > ORC_MAX_STRUCTS) return -1;
    int L = p->levels;
    if (L < 1 || L > ORC_MAX_LEVELS) return -1;
    if (p->contour_level_mask >> L) return -1;
    if (initial_u && L != 1) return -1;
    for (int lv = 0; lv < L; ++lv)
        if (p->iters[lv] < 0) return -1;

    int dims[ORC_MAX_LEVELS][3];
    double *I0[ORC_MAX_LEVELS], *T0[ORC_MAX_LEVELS];
    size_t n0 = (size_t)nx * ny * nz;
    dims[0][0] = nx; dims[0][1] = ny; dims[0][2] = nz;
    I0[0] = (double *)malloc(sizeof(double) * n0);
    T0[0] = (double *)malloc(sizeof(double) * n0);
    memcpy(I0[0], moving, sizeof(double) * n0);
    memcpy(T0[0], target, sizeof(double) * n0);
    /* initialisation: down-sample the images to the coarsest level */
    for (int lv = 1; lv < L; ++lv) {
        for (int a = 0; a < 3; ++a) dims[lv][a] = (dims[lv - 1][a] + 1) / 2;
        size_t nl = (size_t)dims[lv][0] * dims[lv][1] * dims[lv][2];
        I0[lv] = (double *)malloc(sizeof(double) * nl);
        T0[lv] = (double *)malloc(sizeof(double) * nl);
        orc_restrict(I0[lv - 1], dims[lv - 1][0], dims[lv - 1][1], dims[lv - 1][2], p->restrict_sigma, I0[lv]);
        orc_restrict(T0[lv - 1], dims[lv - 1][0], dims[lv - 1][1], dims[lv - 1][2], p->restrict_sigma, T0[lv]);
    }
    /* the structure masks of every level that has contour terms (and of the levels between) */
    const uint8_t *TM[ORC_MAX_LEVELS] = {tmasks}, *MM[ORC_MAX_LEVELS] = {mmasks};
    uint8_t *own_masks[2 * ORC_MAX_LEVELS] = {0};
    int top = 0;
    for (int lv = 1; lv < L; ++lv)
        if ((p->contour_level_mask >> lv) & 1u) top = lv;
    for (int lv = 1; lv <= top && k > 0; ++lv) {
        size_t nl = (size_t)dims[lv][0] * dims[lv][1] * dims[lv][2];
        uint8_t *t = (uint8_t *)malloc((size_t)k * nl), *m = (uint8_t *)malloc((size_t)k * nl);
        orc_decimate_masks(TM[lv - 1], k, dims[lv - 1][0], dims[lv - 1][1], dims[lv - 1][2], t);
        orc_decimate_masks(MM[lv - 1], k, dims[lv - 1][0], dims[lv - 1][1], dims[lv - 1][2], m);
        TM[lv] = own_masks[2 * lv] = t;
        MM[lv] = own_masks[2 * lv + 1] = m;
    }

    /* u0 := 0 at the coarsest level (or the given initial field) */
    size_t nc = (size_t)dims[L - 1][0] * dims[L - 1][1] * dims[L - 1][2];
    double *u = (double *)calloc(3 * nc, sizeof(double));
    if (initial_u) memcpy(u, initial_u, sizeof(double) * 3 * n0);

    /* the stopping region and the signs of the modified images */
    uint8_t *uroi = NULL;
    int sign[ORC_MAX_STRUCTS];
    int want_uroi = (p->stop_mode != 0) || (delta_hist != NULL);
    double *hist = delta_hist;
    if (p->stop_mode && !hist) hist = (double *)calloc((size_t)(p->iters[0] > 0 ? p->iters[0] : 1), sizeof(double));
    if (want_uroi) {
        uroi = (uint8_t *)malloc(n0);
        if (k > 0) orc_uroi(tmasks, k, nx, ny, nz, p->uroi_radius, uroi);
        else memset(uroi, 1, n0);
    }
    for (int s = 0; s < k; ++s)
        sign[s] = p->sign[s] != 0 ? (p->sign[s] > 0 ? 1 : -1)
                                  : orc_auto_sign(T0[0], tmasks + (size_t)s * n0, nx, ny, nz, p->uroi_radius);

    int done = 0;
    for (int lv = L - 1; lv >= 0; --lv) {
        int lx = dims[lv][0], ly = dims[lv][1], lz = dims[lv][2];
        size_t nl = (size_t)lx * ly * lz;
        if (lv < L - 1) { /* up-sample the field to this level */
            double *uf = (double *)malloc(sizeof(double) * 3 * nl);
            orc_prolong(u, dims[lv + 1][0], dims[lv + 1][1], dims[lv + 1][2], lx, ly, lz, uf);
            free(u);
            u = uf;
        }
        int kl = ((p->contour_level_mask >> lv) & 1u) ? k : 0;
        double **Ip = NULL, **Tp = NULL;
        if (kl > 0) { /* create the modified images */
            Ip = (double **)malloc(sizeof(double *) * kl);
            Tp = (double **)malloc(sizeof(double *) * kl);
            for (int s = 0; s < kl; ++s) {
                Ip[s] = (double *)malloc(sizeof(double) * nl);
                Tp[s] = (double *)malloc(sizeof(double) * nl);
                orc_modified_image(I0[lv], MM[lv] + (size_t)s * nl, sign[s], p->c0, nl, Ip[s]);
                orc_modified_image(T0[lv], TM[lv] + (size_t)s * nl, sign[s], p->c0, nl, Tp[s]);
            }
        }
        int fine = (lv == 0);
        int W = p->stop_window > 0 ? p->stop_window : 10;
        /* physical voxel size of this level (the finest size doubles per level), or voxel
           units throughout when no spacing is given */
        double hl[3] = {1.0, 1.0, 1.0};
        if (p->spacing[0] > 0.0)
            for (int a = 0; a < 3; ++a) hl[a] = p->spacing[a] * (double)(1 << lv);
        for (int it = 0; it < p->iters[lv]; ++it) {
            double delta = 0.0;
            int need_delta = fine && want_uroi;
            orc_step(I0[lv], T0[lv], lx, ly, lz, kl, (const double *const *)Ip, (const double *const *)Tp,
                     p->lambda, p->sigma_fluid, p->sigma_diff, hl, need_delta ? uroi : NULL, p->norm_range,
                     u, need_delta ? &delta : NULL);
            if (fine) {
                if (hist) hist[it] = delta;
                done = it + 1;
                /* stopping rule, evaluated after every W iterations */
                if (p->stop_mode && (it + 1) % W == 0 && it - W >= 0 &&
                    hist[it - W] - hist[it] <= p->stop_eps)
                    break;
            }
        }
        if (kl > 0) {
            for (int s = 0; s < kl; ++s) { free(Ip[s]); free(Tp[s]); }
            free(Ip);
            free(Tp);
        }
    }
    memcpy(u_out, u, sizeof(double) * 3 * n0);
    if (iters_done) *iters_done = done;
    free(u);
    free(uroi);
    if (hist != delta_hist) free(hist);
    for (int lv = 0; lv < L; ++lv) { free(I0[lv]); free(T0[lv]); }
    for (int q = 0; q < 2 * ORC_MAX_LEVELS; ++q) free(own_masks[q]);
    return 0;
}
