// HIP kernels of the registration evaluation (section 2.3): intensity agreement of the
// deformed moving image with the target (RMS-ID, CC), volume overlap of the deformed
// structures (DSC), and contour propagation (opening, boundary extraction) with the
// surface-to-surface distance (SSD) of each propagated contour.
//
// Reductions are deterministic: a fixed grid walks the volume in a fixed order, each block
// reduces in a fixed tree, and the host adds the block partials in block order.
#include <hipcub/hipcub.hpp>

#include "cgdir_internal.h"

namespace cgdir {
namespace {

constexpr int kRedBlocks = 512, kRedThreads = 256;

// block sum of NV doubles per thread, in a fixed tree; thread 0 writes the block's partials
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double *out)
{
    __shared__ double sh[NV][kRedThreads];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int q = 0; q < NV; ++q) sh[q][t] += sh[q][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) out[(int64_t)blockIdx.x * NV + q] = sh[q][0];
    }
}

// pass 1: count, sum a, sum b over the volume and over the region
__global__ void __launch_bounds__(kRedThreads) k_intensity_pass1(const float *__restrict__ a,
                                                                 const float *__restrict__ b,
                                                                 const uint8_t *__restrict__ region, int64_t n,
                                                                 double *partials)
{
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const double x = a[i], y = b[i];
        v[0] += 1.0;
        v[1] += x;
        v[2] += y;
        if (region && region[i]) {
            v[3] += 1.0;
            v[4] += x;
            v[5] += y;
        }
    }
    block_sum_store<6>(v, partials);
}

// pass 2: sums of (a - b)^2, (a - ma)^2, (b - mb)^2, (a - ma)(b - mb) over the volume and
// over the region, with the means of pass 1
__global__ void __launch_bounds__(kRedThreads) k_intensity_pass2(const float *__restrict__ a,
                                                                 const float *__restrict__ b,
                                                                 const uint8_t *__restrict__ region, int64_t n,
                                                                 double ma, double mb, double ra, double rb,
                                                                 double *partials)
{
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const double x = a[i], y = b[i];
        const double e = x - y, da = x - ma, db = y - mb;
        v[0] += e * e;
        v[1] += da * da;
        v[2] += db * db;
        v[3] += da * db;
        if (region && region[i]) {
            const double qa = x - ra, qb = y - rb;
            v[4] += e * e;
            v[5] += qa * qa;
            v[6] += qb * qb;
            v[7] += qa * qb;
        }
    }
    block_sum_store<8>(v, partials);
}

// |D|, |T|, |D and T| for one structure; T is bit `bit` of tbits
__global__ void __launch_bounds__(kRedThreads) k_overlap_counts(const uint8_t *__restrict__ D,
                                                                const uint8_t *__restrict__ tbits, int bit,
                                                                int64_t n, double *partials)
{
    double v[3] = {0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const bool d = D[i] != 0, t = (tbits[i] >> bit) & 1u;
        v[0] += d ? 1.0 : 0.0;
        v[1] += t ? 1.0 : 0.0;
        v[2] += (d && t) ? 1.0 : 0.0;
    }
    block_sum_store<3>(v, partials);
}

// sum and sum of squared deviations from `mean` of n values
__global__ void __launch_bounds__(kRedThreads) k_value_sums(const double *__restrict__ x, int64_t n, double mean,
                                                            double *partials)
{
    double v[2] = {0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const double d = x[i] - mean;
        v[0] += x[i];
        v[1] += d * d;
    }
    block_sum_store<2>(v, partials);
}

// Binary morphology with the 6-connected cross; outside the volume counts as outside.
// src is a byte mask (nonzero = inside) or, with bit >= 0, bit `bit` of a bit-plane.
__device__ __forceinline__ bool inside(const uint8_t *__restrict__ m, int bit, int64_t i)
{
    return bit < 0 ? m[i] != 0 : ((m[i] >> bit) & 1u) != 0;
}

// mode 0: erosion (the voxel and its 6 neighbours inside), 1: dilation (any of them inside),
// 2: boundary (inside with a neighbour outside)
__global__ void __launch_bounds__(256) k_cross(const uint8_t *__restrict__ src, int bit, Dims d, int mode,
                                               uint8_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.n()) return;
    const int x = (int)(i % d.nx), y = (int)((i / d.nx) % d.ny), z = (int)(i / ((int64_t)d.nx * d.ny));
    const int64_t sx = 1, sy = d.nx, sz = (int64_t)d.nx * d.ny;
    const bool c = inside(src, bit, i);
    bool all = c, any = c;
    const bool nb[6] = {x > 0 && inside(src, bit, i - sx), x + 1 < d.nx && inside(src, bit, i + sx),
                        y > 0 && inside(src, bit, i - sy), y + 1 < d.ny && inside(src, bit, i + sy),
                        z > 0 && inside(src, bit, i - sz), z + 1 < d.nz && inside(src, bit, i + sz)};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        all = all && nb[q];
        any = any || nb[q];
    }
    dst[i] = mode == 0 ? (uint8_t)all : (mode == 1 ? (uint8_t)any : (uint8_t)(c && !all));
}

// nonzero bytes of a mask
__global__ void __launch_bounds__(kRedThreads) k_count_nonzero(const uint8_t *__restrict__ m, int64_t n,
                                                               double *partials)
{
    double v[1] = {0};
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        v[0] += m[i] ? 1.0 : 0.0;
    block_sum_store<1>(v, partials);
}

// SSD by brute force: for each contour point, the shortest distance (mm) to a surface point.
// Surface points are staged through LDS in tiles; distances ((dx sx)^2 + (dy sy)^2) + (dz sz)^2
// in FP64 with integer voxel offsets, square root of the minimum.
constexpr int kSsdThreads = 256, kSsdTile = 1024;
__global__ void __launch_bounds__(kSsdThreads) k_ssd(const int *__restrict__ cpts, int nc, const int *__restrict__ spts,
                                                     int ns, Dims d, double sx, double sy, double sz,
                                                     double *__restrict__ out)
{
    __shared__ int tile[3][kSsdTile];
    const int p = blockIdx.x * kSsdThreads + threadIdx.x;
    int px = 0, py = 0, pz = 0;
    if (p < nc) {
        const int v = cpts[p];
        px = v % d.nx;
        py = (v / d.nx) % d.ny;
        pz = v / (d.nx * d.ny);
    }
    double best = INFINITY;
    for (int t0 = 0; t0 < ns; t0 += kSsdTile) {
        const int m = min(kSsdTile, ns - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += kSsdThreads) {
            const int v = spts[t0 + q];
            tile[0][q] = v % d.nx;
            tile[1][q] = (v / d.nx) % d.ny;
            tile[2][q] = v / (d.nx * d.ny);
        }
        __syncthreads();
        if (p < nc) {
            for (int q = 0; q < m; ++q) {
                const double ex = (double)(px - tile[0][q]) * sx;
                const double ey = (double)(py - tile[1][q]) * sy;
                const double ez = (double)(pz - tile[2][q]) * sz;
                const double d2 = ex * ex + ey * ey + ez * ez;
                best = d2 < best ? d2 : best;
            }
        }
    }
    if (p < nc) out[p] = sqrt(best);
}

int blocks_of(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

int eval_red_blocks() { return kRedBlocks; }

hipError_t launch_intensity_pass1(const float *a, const float *b, const uint8_t *region, int64_t n, double *partials,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_intensity_pass1, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, region, n, partials);
    return hipGetLastError();
}

hipError_t launch_intensity_pass2(const float *a, const float *b, const uint8_t *region, int64_t n, double ma,
                                  double mb, double ra, double rb, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_intensity_pass2, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, region, n, ma, mb, ra, rb,
                       partials);
    return hipGetLastError();
}

hipError_t launch_overlap_counts(const uint8_t *D, const uint8_t *tbits, int bit, int64_t n, double *partials,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_overlap_counts, dim3(kRedBlocks), dim3(kRedThreads), 0, s, D, tbits, bit, n, partials);
    return hipGetLastError();
}

hipError_t launch_value_sums(const double *x, int64_t n, double mean, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_value_sums, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, n, mean, partials);
    return hipGetLastError();
}

hipError_t launch_cross(const uint8_t *src, int bit, Dims d, int mode, uint8_t *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_cross, dim3(blocks_of(d.n(), 256)), dim3(256), 0, s, src, bit, d, mode, dst);
    return hipGetLastError();
}

hipError_t launch_count_nonzero(const uint8_t *m, int64_t n, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_nonzero, dim3(kRedBlocks), dim3(kRedThreads), 0, s, m, n, partials);
    return hipGetLastError();
}

hipError_t launch_ssd(const int *cpts, int nc, const int *spts, int ns, Dims d, const float spacing[3], double *out,
                      hipStream_t s)
{
    if (nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ssd, dim3(blocks_of(nc, kSsdThreads)), dim3(kSsdThreads), 0, s, cpts, nc, spts, ns, d,
                       (double)spacing[0], (double)spacing[1], (double)spacing[2], out);
    return hipGetLastError();
}

// Linear indices (ascending) of the nonzero bytes of flags: device-wide selection.
hipError_t select_flagged(void *temp, size_t *temp_bytes, const uint8_t *flags, int64_t n, int *out, int *count,
                          hipStream_t s)
{
    hipcub::CountingInputIterator<int> idx(0);
    return hipcub::DeviceSelect::Flagged(temp, *temp_bytes, idx, flags, out, count, (int)n, s);
}

hipError_t sort_doubles(void *temp, size_t *temp_bytes, const double *in, double *out, int n, hipStream_t s)
{
    return hipcub::DeviceRadixSort::SortKeys(temp, *temp_bytes, in, out, n, 0, (int)(8 * sizeof(double)), s);
}

}  // namespace cgdir
