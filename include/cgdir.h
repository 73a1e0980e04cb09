/*
 * libcgdir -- contour-guided demons deformable registration (CG-DIR) on MI355X.
 *
 * Computes the deformation vector field u that registers a moving CT image I0 onto a
 * target CT image T0 (section 2.1, Eq.1: u = argmin 1/2 |I0 o u - T0|^2 + a/2 |grad u|^2)
 * with the contour term of Eq.2: each delineated structure i contributes a pair of
 * modified images I_i = (1 + M_i/2) I0, T_i = (1 + N_i/2) T0 built from its mask on the
 * moving image (M_i) and on the target image (N_i).  The iteration is Algorithm A:
 * a multi-resolution pyramid, plain demons on the coarse levels, and at the finest level
 * the loop {Eq.7 step du along n = grad I0~/|grad I0~| with beta = (T0 - I0~)^2,
 * Gaussian smoothing of du, composite update u <- du + u o (Id + du), Gaussian
 * smoothing of u} (section 2.2).  Arithmetic is FP32 on the GPU.
 *
 * Conventions (every entry point):
 *   - volumes are float32, x fastest: element (i, j, l) at i + nx*(j + ny*l);
 *   - a displacement field is float32 [3][nz][ny][nx]: the x, y, z components (SoA),
 *     in voxel units, on the target grid, such that I0(x + u(x)) ~ T0(x);
 *   - masks are uint8 [nz][ny][nx], 0 = outside, nonzero = inside;
 *   - `where` says whether a buffer is host memory (CGDIR_HOST) or device memory on the
 *     context's device (CGDIR_DEVICE);
 *   - the caller owns every buffer it passes; the library owns only its context and the
 *     sub-allocations it makes inside the pool the caller provides;
 *   - every call returns CGDIR_OK (0) or a negative CGDIR_E_* code; no exception
 *     crosses the boundary; cgdir_strerror() names a code.
 */
#ifndef CGDIR_H
#define CGDIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGDIR_MAX_STRUCTS 8 /* structures per registration (bits of one mask byte) */
#define CGDIR_MAX_LEVELS 6  /* pyramid levels */
#define CGDIR_KEEP_FINISHED 4096 /* served requests whose final status a context keeps */

enum cgdir_code {
    CGDIR_OK = 0,
    CGDIR_E_INVAL = -1,     /* invalid argument (dims, k, pointers, parameters) */
    CGDIR_E_NOMEM = -2,     /* the pool cannot hold the request */
    CGDIR_E_HIP = -3,       /* a HIP runtime call failed */
    CGDIR_E_BUSY = -4,      /* no free serving slot (only from non-queueing calls) */
    CGDIR_E_NOTFOUND = -5,  /* unknown ticket */
    CGDIR_E_CANCELLED = -6, /* the request was cancelled */
    CGDIR_E_NONFINITE = -7, /* the field or the metric became NaN/Inf */
    CGDIR_E_UNIMPL = -8,    /* a parameter combination that is not implemented */
    CGDIR_E_TIMEOUT = -9,   /* cgdir_wait timed out */
    CGDIR_E_SCRATCH = -10   /* cgdir_register_static: the registration needs more device memory
                               than the static scratch holds (CGDIR_STATIC_SCRATCH_BYTES) */
};

/* Device memory of cgdir_register_static, per device (bytes). */
#define CGDIR_STATIC_SCRATCH_BYTES (64u << 20)

enum cgdir_where { CGDIR_HOST = 0, CGDIR_DEVICE = 1 };
enum cgdir_warp_mode { CGDIR_WARP_LINEAR = 0, CGDIR_WARP_MASK = 1 };
enum cgdir_state { CGDIR_QUEUED = 0, CGDIR_RUNNING = 1, CGDIR_DONE = 2, CGDIR_FAILED = 3,
                   CGDIR_CANCELLED = 4 };
enum cgdir_ctx_flags { CGDIR_CTX_PROFILE = 1 /* time every kernel launch with HIP events */ };

typedef struct cgdir_ctx cgdir_ctx;

/* Context description.  `stream` is a hipStream_t on `device` (NULL: the library creates
 * one with default priority).  All of the context's device work runs on that stream and is
 * ordered after nothing else: device inputs written on another stream must be complete (or
 * that stream waited on) before a call reads them.  `pool`/`pool_bytes` is device memory the caller owns and
 * keeps alive until cgdir_destroy returns (pool NULL: the library allocates pool_bytes
 * itself at create time).  Every per-registration buffer is carved out of the pool, so
 * no registration call allocates device memory.  `max_slots` bounds the registrations
 * the serving loop runs concurrently (>= 1). */
typedef struct cgdir_ctx_desc {
    int device;
    void *stream;
    void *pool;
    size_t pool_bytes;
    int max_slots;
    int flags;
} cgdir_ctx_desc;

/* A float32 volume (the moving or the target CT, HU). */
typedef struct cgdir_volume {
    const void *data;
    int nx, ny, nz;
    int where;
} cgdir_volume;

/* k structure masks on one image (section 2.1: O_i^p on the moving image, O_i^t on the
 * target image; the i-th plane of both describes the same structure).  `planes` is a
 * host array of k pointers, each to a uint8 volume of the image's dims. */
typedef struct cgdir_masks {
    int k;
    const uint8_t *const *planes;
    int where;
} cgdir_masks;

/* Parameters (section 2.2).  cgdir_params_default() fills the defaults named here. */
typedef struct cgdir_params {
    int levels;                      /* pyramid levels; default 1.  The paper uses 2 (section 2.2) */
    int iters[CGDIR_MAX_LEVELS];     /* iterations per level, index 0 = finest; default 100 */
    unsigned contour_level_mask;     /* bit l: contour terms at level l; default 1 (finest only,
                                        as in Algorithm A).  At a coarse level l the structure
                                        masks are those of the finest voxels at indices
                                        2^l (i, j, k), the voxels the restriction keeps; bits at
                                        or above `levels` give CGDIR_E_INVAL */
    float sigma_fluid;               /* Gaussian sigma smoothing du (voxels); default 1 */
    float sigma_diff;                /* Gaussian sigma smoothing u (voxels); default 1 */
    float restrict_sigma;            /* Gaussian sigma of the pyramid restriction; default 1 */
    float lambda[CGDIR_MAX_STRUCTS]; /* contour weights; default 1e-3 (section 2.2) */
    int sign[CGDIR_MAX_STRUCTS];     /* sign of M_i, N_i: +1 (structure brighter than its
                                        surroundings) or -1; 0 = decide from the target image */
    float intensity_offset;          /* c0: the modified images scale CT numbers HU + c0;
                                        default 1000 */
    int stop_mode;                   /* 0: run the iteration counts; 1: stopping rule of
                                        section 2.2 at the finest level (see below) */
    float stop_eps;                  /* default 1e-4 */
    int stop_window;                 /* default 10 */
    float norm_range;                /* delta = RMS over the UROI of (T0 - I0~)/norm_range;
                                        default 2500 HU */
    int uroi_margin[3];              /* UROI: target structures dilated by an ellipsoid with
                                        these semi-axes (voxels); default {5, 5, 4} = 1 cm at
                                        1.97 x 1.97 x 2.5 mm voxels */
    const float *initial_dvf;        /* optional [3][nz][ny][nx] field to start the finest level
                                        from; then levels must be 1 (section 4: warm start) */
    int initial_dvf_where;
    double *delta_hist;              /* optional host output: delta at each finest-level
                                        iteration (capacity iters[0]) */
    int *iters_done;                 /* optional host output: finest-level iterations run */
    float spacing[3];                /* voxel size of the finest level along x, y, z (e.g. mm,
                                        1.97, 1.97, 2.5 in section 2.3); {0, 0, 0} (default) =
                                        voxel units at every level.  With a spacing the
                                        gradients are per unit length, the step of Eq.7 is in
                                        that unit (converted to voxels for the field),
                                        sigma_fluid and sigma_diff are in that unit (sigma / h
                                        voxels along each axis, radius ceil(3 sigma / h) <= 6),
                                        and level l has voxel size spacing * 2^l; the three
                                        axes may differ.  restrict_sigma and uroi_margin stay
                                        in voxels. */
} cgdir_params;

/* Stopping rule (section 2.2, delta = RMS intensity difference over the UROI, l = change of
 * delta): the finest level stops after iteration n when (n + 1) is a multiple of
 * stop_window, n >= stop_window and delta_{n - stop_window} - delta_n <= stop_eps.  The rule
 * is evaluated on the device, inside the kernel that reduces delta; the launches of later
 * iterations then do nothing for that registration, and the host learns of the stop from
 * a non-blocking copy every stop_window iterations (no host round trip on the path). */

void cgdir_params_default(cgdir_params *p);

/* Create a context on desc->device.  Returns CGDIR_E_INVAL for a bad description,
 * CGDIR_E_HIP if the device cannot be used, CGDIR_E_NOMEM if pool is NULL and
 * pool_bytes cannot be allocated. */
int cgdir_create(cgdir_ctx **out, const cgdir_ctx_desc *desc);

/* Cancel queued requests, wait for running ones, release the context (not the pool). */
int cgdir_destroy(cgdir_ctx *ctx);

/* Register one pair, blocking (Algorithm A).  target and moving have the same dims
 * (each >= 1, at most 4096).  target_masks and moving_masks have the same k
 * (0 <= k <= CGDIR_MAX_STRUCTS; k = 0 is plain demons) and the image's dims; may be NULL
 * for k = 0.  dvf_out receives u, [3][nz][ny][nx] float32 at dvf_where.
 * Returns after dvf_out is written.  Inputs are read in place when on the device.
 * Errors: CGDIR_E_INVAL (dims, k, pointers, parameters), CGDIR_E_NOMEM (the pool cannot
 * hold cgdir_footprint() bytes), CGDIR_E_NONFINITE (non-finite inputs produced a
 * non-finite field), CGDIR_E_HIP. */
int cgdir_register(cgdir_ctx *ctx, const cgdir_volume *target, const cgdir_volume *moving,
                   const cgdir_masks *target_masks, const cgdir_masks *moving_masks,
                   const cgdir_params *params, float *dvf_out, int dvf_where);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid it): cgdir_register on device buffers that allocates nothing.
 * Its per-registration buffers come from a static device array of CGDIR_STATIC_SCRATCH_BYTES
 * (64 MiB) that each device holds until the process ends, instead of the context pool; the
 * context must have been created (cgdir_create looks the array up on its device) and its own
 * stream runs the work.  The call creates no events and makes no memset: what must start at
 * zero is cleared by fill kernels.  Every call on one device shares that device's array, which
 * keeps the last call's contents; calls that overlap on one device would race, so the library
 * runs them one at a time per device (a lock), and nothing else may use the array.
 * Arguments as cgdir_register, with every buffer on the device (CGDIR_E_INVAL otherwise).
 * Limits: about 36 bytes per voxel with contour terms (up to about 1.8 M voxels),
 * CGDIR_E_SCRATCH beyond; the stopping rule, delta_hist and automatic signs (sign 0) need
 * host records and copies and give CGDIR_E_UNIMPL.  Tile shapes are those the context's
 * autotuner has settled for the launch's group (by earlier cgdir_register calls or
 * cgdir_tuning_import), else the first candidate; no candidate is timed.  Results equal
 * cgdir_register's bit for bit.  Blocking. */
int cgdir_register_static(cgdir_ctx *ctx, const cgdir_volume *target, const cgdir_volume *moving,
                          const cgdir_masks *target_masks, const cgdir_masks *moving_masks,
                          const cgdir_params *params, float *dvf_out);

/* Warp src with a field on src's grid: out(x) = src(x + dvf(x)), trilinear, sample
 * position clamped to the volume (the interpolation of section 2.2, kernel 4).
 * CGDIR_WARP_LINEAR: src and out float32.  CGDIR_WARP_MASK: src and out uint8; the
 * trilinear value of the 0/1 mask, inside when >= 0.5 (propagation of a structure,
 * section 2.3).  dvf and out have src->where's placement.  Blocking. */
int cgdir_warp(cgdir_ctx *ctx, const cgdir_volume *src, const float *dvf, int mode, void *out);

/* One registration request for the batched and served paths: the arguments of
 * cgdir_register.  Every buffer must stay valid and unmodified until the request
 * reaches a final state; the library does not copy them at submit. */
typedef struct cgdir_request {
    cgdir_volume target;
    cgdir_volume moving;
    cgdir_masks target_masks;
    cgdir_masks moving_masks;
    cgdir_params params;
    float *dvf_out;
    int dvf_where;
} cgdir_request;

/* Register n pairs of uneven sizes and structure counts together on the device
 * (blocking): every iteration phase runs once for all pairs of a Gaussian radius that still
 * have work, one launch over all their tiles (CGDIR_BATCH_LANES=2 in the environment spreads
 * the radius groups over two streams of the context that share the device).
 * Each pair's result equals what cgdir_register returns for it alone.  status (host,
 * n entries, may be NULL) receives each pair's code.  Returns the first failing code.
 * Errors: as cgdir_register; CGDIR_E_NOMEM when the pool cannot hold all pairs at once. */
int cgdir_register_batch(cgdir_ctx *ctx, int n, const cgdir_request *reqs, int *status);

/* Serving: queue a request, non-blocking.  Requests are admitted in arrival order when a
 * slot is free and the pool holds their footprint, and new ones join between iterations
 * (continuous batching).  Admitted requests advance iteration by iteration in lockstep groups,
 * their launches merged, on two streams of the context that share the device: the small
 * requests (finest level below 8 M voxels) in one, the large ones in the other, so that a small
 * request does not advance at the pace of a large one's launches; while no request waits for
 * admission the large ones run one at a time, oldest first, and while requests wait all run
 * together.  Device inputs the caller ordered on the context stream before the call are
 * complete before the request reads them.
 * Returns CGDIR_E_NOMEM at once if the footprint exceeds the whole pool, CGDIR_E_INVAL
 * for invalid arguments.  *ticket identifies the request.  A context keeps the status of
 * its CGDIR_KEEP_FINISHED most recently finished requests (done, failed or cancelled); an
 * older ticket is then unknown to cgdir_poll / cgdir_wait / cgdir_cancel. */
int cgdir_submit(cgdir_ctx *ctx, const cgdir_request *req, uint64_t *ticket);

typedef struct cgdir_status {
    int state;           /* enum cgdir_state */
    int error;           /* final code when DONE / FAILED / CANCELLED */
    int level;           /* current pyramid level */
    int iter;            /* iterations done at that level */
    double last_delta;   /* latest delta (when computed) */
    int64_t t_submit_ns; /* steady-clock timestamps */
    int64_t t_admit_ns;
    int64_t t_done_ns;
} cgdir_status;

/* Non-blocking status of a ticket.  CGDIR_E_NOTFOUND for an unknown ticket. */
int cgdir_poll(cgdir_ctx *ctx, uint64_t ticket, cgdir_status *st);

/* Cancel a queued request (a running one finishes).  CGDIR_E_NOTFOUND, or CGDIR_E_BUSY
 * when it is already running or finished. */
int cgdir_cancel(cgdir_ctx *ctx, uint64_t ticket);

/* Wait until the request is final or timeout_ns elapses (< 0: forever).
 * Returns the request's final code, CGDIR_E_TIMEOUT or CGDIR_E_NOTFOUND. */
int cgdir_wait(cgdir_ctx *ctx, uint64_t ticket, int64_t timeout_ns);

/* Pool bytes one registration of this size reserves (admission uses it). */
size_t cgdir_footprint(int nx, int ny, int nz, int k, const cgdir_params *params);

/* Static name of a code. */
const char *cgdir_strerror(int code);

/* Per-kernel timing, filled when the context was created with CGDIR_CTX_PROFILE:
 * launches, summed duration (HIP events on the context stream) and voxels processed of
 * each kernel since the last reset.  Kernels of the iteration are reported per pyramid
 * level as "<kernel>@L<level>" (L0 = finest); set-up kernels by name alone.
 * Returns the number of entries written (<= cap). */
typedef struct cgdir_kernel_stat {
    char name[48];
    int64_t launches;
    double total_ms;
    double voxels;       /* voxels processed by those launches */
} cgdir_kernel_stat;
int cgdir_kernel_stats(cgdir_ctx *ctx, cgdir_kernel_stat *out, int cap, int reset);

/* Tile-shape tuning (the batching of many pairs, one launch per phase, with tile shapes the
 * context picks by timing candidates on their first launches).  A tuning group is one kernel
 * (step or smoothing), its Gaussian radius, the dims of the largest pair in the launch and
 * log2 of the launch's voxel count; results never depend on the shape chosen.
 *
 * cgdir_tuning_export writes the groups that have settled as text, one line per group,
 * "<group> <rows per tile> <planes per tile>\n", NUL-terminated, into buf (cap bytes) and
 * sets *len to the bytes needed including the NUL; buf may be NULL (cap 0) to ask for *len.
 * CGDIR_E_INVAL if cap is too small (nothing written) or len is NULL.
 *
 * cgdir_tuning_import settles groups from such text (for example one exported by an earlier
 * process on the same GPU), so that their launches use those shapes without timing any
 * candidate; later imports of a group replace earlier ones.  CGDIR_E_INVAL, with nothing
 * imported, if a line is malformed or names a shape that is not a candidate of its kernel. */
int cgdir_tuning_export(cgdir_ctx *ctx, char *buf, size_t cap, size_t *len);
int cgdir_tuning_import(cgdir_ctx *ctx, const char *text);

/* ---- evaluation of a registration result (section 2.3) ----------------------------------
 * The paper assesses a field three ways, all computed here on the device:
 *  - intensity: RMS-ID = sqrt(mean((I0~ - T0)^2)) and Pearson's correlation coefficient CC
 *    between the deformed moving image I0~ = I0 o u (trilinear, clamped) and the target, over
 *    the whole volume and over the UROI (target structures dilated by uroi_margin);
 *  - volume overlap: DSC = 2 |V_D and V_T| / (|V_D| + |V_T|) with V_D the deformed structure
 *    (mask warp, as CGDIR_WARP_MASK) and V_T the target structure;
 *  - contours, by volume deformation: V_D is opened (opening_radius erosions, then as many
 *    dilations, by the 6-connected cross; outside the volume counts as outside) to remove
 *    small islands, and its boundary (voxels with a face neighbour outside the set) is the
 *    propagated contour.  SSD of a contour voxel = shortest Euclidean distance in mm to a
 *    voxel of the target surface (the boundary of V_T), voxel centres scaled by spacing;
 *    reported as mean, standard deviation (population) and 95th percentile (linear
 *    interpolation between order statistics). */
typedef struct cgdir_eval_params {
    float spacing[3];    /* voxel size in mm along x, y, z; default 1.97, 1.97, 2.5 */
    int opening_radius;  /* 0..16; default 1 */
    int uroi_margin[3];  /* 0..8 voxels per axis; default {5, 5, 4} */
} cgdir_eval_params;

typedef struct cgdir_eval {
    double rms_id, cc;             /* whole volume (HU; dimensionless) */
    double rms_id_uroi, cc_uroi;   /* over the UROI; NaN when k = 0 */
    int64_t voxels, uroi_voxels;
    int k;
    int64_t deformed_voxels[CGDIR_MAX_STRUCTS];  /* |V_D| */
    int64_t target_voxels[CGDIR_MAX_STRUCTS];    /* |V_T| */
    int64_t overlap_voxels[CGDIR_MAX_STRUCTS];   /* |V_D and V_T| */
    double dsc[CGDIR_MAX_STRUCTS];               /* NaN when both volumes are empty */
    int64_t contour_points[CGDIR_MAX_STRUCTS];   /* voxels of the propagated contour */
    int64_t surface_points[CGDIR_MAX_STRUCTS];   /* voxels of the target surface */
    double ssd_mean[CGDIR_MAX_STRUCTS];          /* mm; NaN when a contour or surface is empty */
    double ssd_sd[CGDIR_MAX_STRUCTS];
    double ssd_p95[CGDIR_MAX_STRUCTS];
} cgdir_eval;

void cgdir_eval_params_default(cgdir_eval_params *ep);

/* Evaluate the field dvf ([3][nz][ny][nx] FP32, voxel units, target grid, host or device per
 * dvf_where) that registers `moving` to `target` (same dims).  Masks as in cgdir_register
 * (k may be 0: intensity metrics only).  Blocking; serialises with the context's other
 * launches; scratch (about 12 bytes per voxel plus the contour point lists, and copies of
 * host inputs) comes from the context pool and is released before return.  The caller owns
 * every buffer.  Errors: CGDIR_E_INVAL (arguments), CGDIR_E_NOMEM (pool), CGDIR_E_HIP. */
int cgdir_evaluate(cgdir_ctx *ctx, const cgdir_volume *target, const cgdir_volume *moving,
                   const cgdir_masks *target_masks, const cgdir_masks *moving_masks,
                   const float *dvf, int dvf_where, const cgdir_eval_params *ep, cgdir_eval *out);

#ifdef __cplusplus
}
#endif
#endif
