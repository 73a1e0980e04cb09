/*
 * FP64 CPU oracle for contour-guided demons registration (CG-DIR).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, literal implementation of what
 * the registration computes, written from the paper's equations and its Algorithm A.
 * It exists to check the HIP library; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Conventions
 *   volumes   double[nz][ny][nx], x fastest: index i + nx*(j + ny*l)
 *   fields    three such planes (x, y, z components), voxel units, target grid
 *   masks     uint8[k][nz][ny][nx], nonzero = inside
 * Every function returns 0 on success and a negative value on invalid arguments.
 *
 * Parity unpinned (no number in the paper tests them; the oracle and the HIP path
 * implement the same written reading): the CT-number offset c0 of the modified
 * images, the pyramid filter, the UROI structuring element, the stopping rule,
 * every border convention (index clamping) and the choice of the masks at coarse levels
 * (the paper's Algorithm A uses none there).
 */
#ifndef CGDIR_ORACLE_H
#define CGDIR_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_STRUCTS 32
#define ORC_MAX_LEVELS 8

typedef struct orc_params {
    int levels;                       /* pyramid levels, >= 1 */
    int iters[ORC_MAX_LEVELS];        /* iterations per level, index 0 = finest */
    unsigned contour_level_mask;      /* bit l: contour terms active at level l (l < levels);
                                         at a coarse level the masks are those of
                                         orc_decimate_masks applied l times */
    double sigma_fluid;               /* Gaussian sigma applied to du (voxels) */
    double sigma_diff;                /* Gaussian sigma applied to u (voxels) */
    double restrict_sigma;            /* Gaussian sigma of the pyramid restriction */
    double lambda[ORC_MAX_STRUCTS];   /* contour weights lambda_i */
    int sign[ORC_MAX_STRUCTS];        /* +1 / -1, or 0 = decide from the target image */
    double c0;                        /* CT-number offset of the modified images (HU) */
    int stop_mode;                    /* 0 = fixed iteration counts, 1 = UROI rule */
    double stop_eps;                  /* epsilon of the stopping rule (normalised units) */
    int stop_window;                  /* window of the stopping rule (iterations) */
    double norm_range;                /* intensity range that normalises delta (HU) */
    int uroi_radius[3];               /* UROI margin, semi-axes in voxels (x, y, z) */
    double spacing[3];                /* voxel size of the finest level (e.g. mm) along x, y, z;
                                         0 = voxel units at every level.  With a spacing,
                                         gradients, the step of Eq.7 and the Gaussian sigmas
                                         are in that unit, at level l the voxel size is
                                         spacing * 2^l, and the field stays in voxels */
} orc_params;

/* Gaussian regulariser (section 2.2): sampled Gaussian of radius ceil(3 sigma),
 * normalised to sum 1.  Returns the radius; w must hold 2R+1 values. */
int orc_gauss_radius(double sigma);
int orc_gauss_weights(double sigma, double *w);
/* Separable 3D Gaussian, x then y then z, clamped indices. out may not alias f. */
int orc_smooth(const double *f, int nx, int ny, int nz, double sigma, double *out);
/* The same with its own sigma (voxels) along x, y and z. */
int orc_smooth_axes(const double *f, int nx, int ny, int nz, const double sigma[3], double *out);

/* Trilinear sample of f at position (px, py, pz), position clamped to the volume. */
double orc_sample(const double *f, int nx, int ny, int nz, double px, double py, double pz);
/* out(x) = f(x + u(x))  (pull-back warp on the target grid). */
int orc_warp(const double *f, int nx, int ny, int nz, const double *u, double *out);
/* mask warp: trilinear of the 0/1 mask, inside when >= 0.5 */
int orc_warp_mask(const uint8_t *m, int nx, int ny, int nz, const double *u, uint8_t *out);
/* Central differences with clamped indices: g = 3 planes. */
int orc_gradient(const double *f, int nx, int ny, int nz, double *g);
/* The same divided by the voxel size h[3] of each axis (h NULL: 1). */
int orc_gradient_h(const double *f, int nx, int ny, int nz, const double *h, double *g);
/* u_c(x) = du(x) + u(x + du(x)), per component. */
int orc_compose(const double *u, const double *du, int nx, int ny, int nz, double *uc);
/* R(F)(j) = (G_sigma * F)(2j); coarse dims ceil(n/2). */
int orc_restrict(const double *f, int nx, int ny, int nz, double sigma, double *out);
/* Structure masks at the next coarser level, where Algorithm A's variant with contour terms
 * below the finest level needs them: a coarse voxel is inside when the fine voxel it stands
 * for (even indices, as the restriction keeps) is inside.  m, out: k masks; coarse dims
 * ceil(n/2). */
int orc_decimate_masks(const uint8_t *m, int k, int nx, int ny, int nz, uint8_t *out);
/* u_f(x) = 2 u_c(x / 2) trilinear; coarse dims must be ceil(fine/2). */
int orc_prolong(const double *uc, int cnx, int cny, int cnz, int fnx, int fny, int fnz,
                double *uf);
/* UROI: union of the target masks dilated by an ellipsoid of semi-axes r (ball painting). */
int orc_uroi(const uint8_t *masks, int k, int nx, int ny, int nz, const int r[3], uint8_t *out);
/* Sign of structure i: +1 when the mean target intensity inside the structure is not
 * lower than in its margin shell (the dilated structure minus itself), else -1. */
int orc_auto_sign(const double *T0, const uint8_t *mask, int nx, int ny, int nz, const int r[3]);
/* Modified image (1 + s/2 * m) * (F + c0). */
int orc_modified_image(const double *F, const uint8_t *mask, int s, double c0, size_t n,
                       double *out);

/* Eq.7 at one voxel.  a0, d: main term; a[i], di[i]: contour terms (already projected on n);
 * returns v.  Requires a0 > 0. */
double orc_eq7(double a0, double d, int k, const double *lambda, const double *a, const double *di);

/* Displacement du of one iteration from warped images (Eq.7 with n = grad I0~ / |grad I0~|). */
int orc_force(const double *wI0, const double *T0, int k, const double *const *wIp,
              const double *const *Tp, const double *lambda, int nx, int ny, int nz,
              double *du);
/* The same with gradients in the unit of the voxel size h[3] (h NULL: voxels): Eq.7 gives a
 * step in that unit, returned converted to voxels (component a divided by h[a]). */
int orc_force_h(const double *wI0, const double *T0, int k, const double *const *wIp,
                const double *const *Tp, const double *lambda, int nx, int ny, int nz,
                const double *h, double *du);

/* One iteration of the loop of Algorithm A at one level: warp, gradient, Eq.7, smooth du,
 * composite update, smooth u.  Iplus/Tplus are the k materialised modified images.
 * h (NULL: voxel units): voxel size; gradients, the step and sigma_f, sigma_d in its unit.
 * If delta != NULL and uroi != NULL, *delta = RMS over the UROI of (T0 - I0~) / norm_range,
 * computed from u before the update.  u is updated in place. */
int orc_step(const double *I0, const double *T0, int nx, int ny, int nz, int k,
             const double *const *Iplus, const double *const *Tplus, const double *lambda,
             double sigma_f, double sigma_d, const double *h, const uint8_t *uroi, double norm_range,
             double *u, double *delta);

/* Algorithm A: pyramid, demons at coarse levels, CG-DIR at the finest level.
 * target/moving: double[N]; masks: uint8[k][N].  initial_u (3N or NULL): start the
 * finest level from it and skip the coarse levels (levels must then be 1).
 * u_out: 3N.  delta_hist (iters[0] or NULL): delta at each finest-level iteration.
 * iters_done (or NULL): finest-level iterations actually run. */
int orc_register(const double *target, const double *moving, int nx, int ny, int nz, int k,
                 const uint8_t *tmasks, const uint8_t *mmasks, const orc_params *p,
                 const double *initial_u, double *u_out, double *delta_hist, int *iters_done);

#ifdef __cplusplus
}
#endif
#endif
