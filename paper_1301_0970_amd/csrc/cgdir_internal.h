// Internal declarations shared by the HIP kernels and the host runtime of libcgdir.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cgdir {

constexpr int kMaxStructs = 8;
constexpr int kMaxRadius = 6;       // Gaussian radius ceil(3 sigma) <= 6  (sigma <= 2)
constexpr int kTileX = 64;          // one wavefront spans a tile row
constexpr int kComputeUnits = 256;  // of an MI355X (8 XCDs x 32)
constexpr int kMaxUroiMargin = 8;

// Geometry of one volume.
struct Dims {
    int nx, ny, nz;
    __host__ __device__ int64_t n() const { return (int64_t)nx * ny * nz; }
};

// The warp of the moving image with the current field (kernel 4 on images):
// I0~(x) = I0(x + u(x)); F(x) = OR of the moving-mask bits at the 8 corners of x's trilinear
// stencil; where F has exactly one bit i, K(x) = (m_i (I0 + c0))(x + u(x)) (elsewhere K is
// neither written nor read).
struct WarpArgs {
    const float *I0;          // moving image at this level
    const uint8_t *mbits;     // moving-mask bits (null: no contour terms at this level)
    const uint8_t *mocc;      // moving-mask occupancy of 8x8x8 bricks (brick_dims)
    float *wI0;
    uint8_t *F;
    float *K;
    Dims d;
    int bnx, bny;             // brick grid x, y extents
    float c0;                 // CT-number offset
};

// Arguments of the step kernel: the force (gradient, Eq.7) on the warped image of the
// current field, its smoothing with sigma_fluid, the composite update u_c = s + u o (Id + s)
// with s the smoothed step, and the stopping-metric partials.
struct StepArgs {
    const float *wI0;         // I0~ of the current field
    const uint8_t *F;         // stencil structure bits (null: k = 0 at this level)
    const float *K;           // K_i~ where F has one bit
    const float *T0;          // target image at this level
    const uint8_t *tbits;     // bit i = voxel inside structure i on the target image
    const uint8_t *uroi;      // stopping region (or null: no metric)
    const float *I0;          // moving image and mask bits: re-warp where several
    const uint8_t *mbits;     //   structures meet in one stencil
    const float *u[3];        // current field
    float *uc[3];             // output: composite update
    float *partials;          // sums of ((T0 - I0~)/norm)^2 over the UROI, one per 64-voxel
                              // row segment: index (z * ny + y) * ceil(nx / 64) + x / 64
    Dims d;
    int k;                    // active structures (<= kMaxStructs)
    float lam[kMaxStructs];   // lambda_i
    float far_l1;             // 1 + lambda_0 + ... + lambda_{k-1}, summed in this order
    float far_c[3];           // 2 far_l1 gs[a]^2 per axis
    float gs2[3];             // gs[a]^2
    uint32_t neg;             // bit i: s_i = -1 (else +1); the modified images use s_i / 2
    float c0;                 // CT-number offset
    float inv_norm;           // 1 / norm_range
    float gs[3];              // 0.5 / voxel size along x, y and z (0.5 in voxel units): central
                              // differences per unit length; the step goes back to voxels as
                              // 2 gs
    // fluid Gaussian along x, y and z: w[0] centre, w[m] = weight at +-m, zero past the
    // axis' own radius (the launch's radius is the largest of the three)
    float wx[kMaxRadius + 1], wy[kMaxRadius + 1], wz[kMaxRadius + 1];
    int tz;                   // planes per block (z chunk)
    const int *stop;          // iterations after which the pair stopped (0: running)
    int iter;                 // this launch's iteration: nothing to do once *stop <= iter
};

// Arguments of the smoothing of u_c into u (diffusion Gaussian), followed by the warp of I0
// with the new u.
struct SmoothArgs {
    const float *in[3];
    float *out[3];
    Dims d;
    // Gaussian along x, y and z: w[0] centre, w[m] = weight at +-m, zero past the axis' radius
    float wx[kMaxRadius + 1], wy[kMaxRadius + 1], wz[kMaxRadius + 1];
    int tz;
    WarpArgs warp;            // where the warp goes
    const int *stop;          // iterations after which the pair stopped (0: running)
    int iter;                 // this launch's iteration: nothing to do once *stop <= iter
};

// One pair's stopping-metric reduction in a batched finalize.
// delta_n = sqrt(sum of partials / count) goes to hist[n].  With window > 0 the stopping
// rule is applied on the device: after iteration n with (n + 1) % window == 0 and
// n >= window, the pair stops when hist[n - window] - delta_n <= eps, and *stop receives
// n + 1 (the iterations run).  Once *stop is set nothing more is recorded.
struct DeltaJob {
    const float *partials;
    int nparts;
    int n;
    const int64_t *count;
    double *hist;
    int *stop;
    double eps;
    int window;
};

// Batched launches: one launch over the tiles of n pairs.  The descriptors travel in the
// kernel-argument segment (<= 4 KiB), so a launch holds a bounded number of pairs.
// prefix[q] = first block of pair q, prefix[n] = total blocks.
constexpr int kBatchStep = 12, kBatchSmooth = 16, kBatchDelta = 64;
struct StepBatch {
    int n;
    int prefix[kBatchStep + 1];
    StepArgs d[kBatchStep];
};
struct SmoothBatch {
    int n;
    int prefix[kBatchSmooth + 1];
    SmoothArgs d[kBatchSmooth];
};
struct DeltaBatch {
    int n;
    DeltaJob d[kBatchDelta];
};
static_assert(sizeof(StepBatch) <= 4096 && sizeof(SmoothBatch) <= 4096 && sizeof(DeltaBatch) <= 4096,
              "kernel arguments are limited to 4 KiB");

// ---- launchers (cgdir_kernels.hip); each returns the hipError_t of its launch -------
hipError_t launch_step_batch(const StepBatch &b, int radius, int ty, hipStream_t s);
hipError_t launch_smooth_batch(const SmoothBatch &b, int radius, int ty, hipStream_t s);
hipError_t launch_delta_batch(const DeltaBatch &b, hipStream_t s);
hipError_t launch_warp_init(const WarpArgs &w, const float *const u[3], hipStream_t s);
int tile_blocks(Dims d, int ty, int tz);
hipError_t launch_brick_occupancy(const uint8_t *bits, Dims d, uint8_t *occ, hipStream_t s);
hipError_t launch_restrict_pass(const float *in, float *out, Dims din, int axis, const float *w,
                                int radius, hipStream_t s);
hipError_t launch_prolong(const float *const uc[3], Dims dc, float *const uf[3], Dims df,
                          hipStream_t s);
hipError_t launch_pack_masks(const uint8_t *const *planes, int k, int64_t n, uint8_t *bits,
                             hipStream_t s);
hipError_t launch_level_bits(const uint8_t *bits0, Dims d0, int level, uint8_t *out, Dims dc, hipStream_t s);
hipError_t launch_uroi(const uint8_t *tbits, Dims d, const int margin[3], uint8_t *rowdist,
                       uint8_t *uroi, hipStream_t s);
hipError_t launch_count(const uint8_t *m, int64_t n, uint8_t bitmask, int64_t *partials,
                        int *nparts, int64_t *out, hipStream_t s);
hipError_t launch_warp_linear(const float *src, Dims d, const float *const u[3], float *out,
                              hipStream_t s);
hipError_t launch_warp_mask(const uint8_t *src, Dims d, const float *const u[3], uint8_t *out,
                            hipStream_t s);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_nonfinite(const float *p, int64_t n, int *flag, hipStream_t s);
hipError_t launch_sign_stats(const float *T0, const uint8_t *tbits, const uint8_t *dil, int bit,
                             int64_t n, double *partials, int *nparts, double *out4,
                             hipStream_t s);
hipError_t launch_dilate_bit(const uint8_t *bits, int bit, Dims d, const int margin[3],
                             uint8_t *rowdist, uint8_t *out, hipStream_t s);


// evaluation (cgdir_eval.hip): reductions write eval_red_blocks() block partials of NV
// doubles each, added by the host in block order
int eval_red_blocks();
hipError_t launch_intensity_pass1(const float *a, const float *b, const uint8_t *region, int64_t n,
                                  double *partials, hipStream_t s);  // NV = 6
hipError_t launch_intensity_pass2(const float *a, const float *b, const uint8_t *region, int64_t n, double ma,
                                  double mb, double ra, double rb, double *partials, hipStream_t s);  // NV = 8
hipError_t launch_overlap_counts(const uint8_t *D, const uint8_t *tbits, int bit, int64_t n, double *partials,
                                 hipStream_t s);  // NV = 3
hipError_t launch_value_sums(const double *x, int64_t n, double mean, double *partials, hipStream_t s);  // NV = 2
hipError_t launch_count_nonzero(const uint8_t *m, int64_t n, double *partials, hipStream_t s);  // NV = 1
// mode 0 erosion, 1 dilation, 2 boundary, by the 6-connected cross; bit >= 0 reads a bit-plane
hipError_t launch_cross(const uint8_t *src, int bit, Dims d, int mode, uint8_t *dst, hipStream_t s);
hipError_t launch_ssd(const int *cpts, int nc, const int *spts, int ns, Dims d, const float spacing[3], double *out,
                      hipStream_t s);
// temp == nullptr: *temp_bytes receives the scratch size needed
hipError_t select_flagged(void *temp, size_t *temp_bytes, const uint8_t *flags, int64_t n, int *out, int *count,
                          hipStream_t s);
hipError_t sort_doubles(void *temp, size_t *temp_bytes, const double *in, double *out, int n, hipStream_t s);

// row-segment partials of the stopping metric for a volume
inline int64_t metric_parts(Dims d) { return (int64_t)((d.nx + kTileX - 1) / kTileX) * d.ny * d.nz; }

// brick grid of the mask occupancy map (8x8x8 voxels per brick)
inline Dims brick_dims(Dims d) { return Dims{(d.nx + 7) / 8, (d.ny + 7) / 8, (d.nz + 7) / 8}; }

}  // namespace cgdir
