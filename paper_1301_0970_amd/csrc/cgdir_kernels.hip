// HIP kernels of libcgdir for gfx950 (MI355X): the per-voxel CG-DIR iteration
// (section 2.1, Eqs. 5-7; section 2.2, the five data-parallel kernels) and its
// pyramid / mask / metric helpers.  FP32 arithmetic, x-fastest volumes, SoA fields.
//
// Every per-voxel result depends only on the voxel and the data, never on the tile
// shape or on what else shares the launch, so results are bitwise reproducible
// whether a pair runs alone or batched.
#include <math.h>

#include "cgdir_internal.h"

namespace cgdir {
namespace {

__device__ __forceinline__ float lerpf(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Sample coordinate p = i + u on an axis of n voxels, clamped to [0, n-1] (trilinear
// interpolation with replicated borders): base index, successor and fraction.  The
// coordinate is split into integer and fractional parts so that i + u is never rounded.
struct Split {
    int i0, i1;
    float t;
};

__device__ __forceinline__ Split split_axis(int i, float u, int n)
{
    const float fu = floorf(u);
    float t = u - fu;
    const float pb = (float)i + fu;
    Split s;
    if (pb < 0.f) {
        s.i0 = 0;
        t = 0.f;
    } else if (pb >= (float)(n - 1)) {
        s.i0 = n - 1;
        t = 0.f;
    } else {
        s.i0 = (pb == pb) ? (int)pb : 0;  // NaN keeps an in-bounds index and a NaN weight
    }
    s.i1 = min(s.i0 + 1, n - 1);
    s.t = t;
    return s;
}

// Corner offsets of a trilinear stencil: row bases for (y0,z0), (y1,z0), (y0,z1), (y1,z1).
struct Corners {
    int r00, r10, r01, r11, x0, x1;
    float tx, ty, tz;
};

__device__ __forceinline__ Corners corners(const Split &sx, const Split &sy, const Split &sz, int nx,
                                           int nxy)
{
    Corners c;
    c.r00 = sy.i0 * nx + sz.i0 * nxy;
    c.r10 = sy.i1 * nx + sz.i0 * nxy;
    c.r01 = sy.i0 * nx + sz.i1 * nxy;
    c.r11 = sy.i1 * nx + sz.i1 * nxy;
    c.x0 = sx.i0;
    c.x1 = sx.i1;
    c.tx = sx.t;
    c.ty = sy.t;
    c.tz = sz.t;
    return c;
}

// lerp in x, then y, then z of the 8 corner values f[0..7] ordered
// (x0,y0,z0) (x1,y0,z0) (x0,y1,z0) (x1,y1,z0) (x0,y0,z1) (x1,y0,z1) (x0,y1,z1) (x1,y1,z1)
__device__ __forceinline__ float lerp8(const float f[8], float tx, float ty, float tz)
{
    const float c00 = lerpf(f[0], f[1], tx);
    const float c10 = lerpf(f[2], f[3], tx);
    const float c01 = lerpf(f[4], f[5], tx);
    const float c11 = lerpf(f[6], f[7], tx);
    return lerpf(lerpf(c00, c10, ty), lerpf(c01, c11, ty), tz);
}

__device__ __forceinline__ float trilinear(const float *__restrict__ f, const Corners &c)
{
    float v[8];
    v[0] = f[c.r00 + c.x0];
    v[1] = f[c.r00 + c.x1];
    v[2] = f[c.r10 + c.x0];
    v[3] = f[c.r10 + c.x1];
    v[4] = f[c.r01 + c.x0];
    v[5] = f[c.r01 + c.x1];
    v[6] = f[c.r11 + c.x0];
    v[7] = f[c.r11 + c.x1];
    return lerp8(v, c.tx, c.ty, c.tz);
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// ============================================================================
// Force: kernels 2 (gradient), 3 (moving vector, Eq.7) and the image half of kernel 4
// (warp) fused.  A block owns a 64 x TY column tile and marches through a chunk of z
// planes.  The warped moving image I0~ = I0(x + u) and the warped masked images
// K_i~ = (m_i (I0 + c0))(x + u) of each plane (tile + 1-voxel halo) go to a 3-plane LDS
// ring, from which the central differences are taken.  With s_i the sign of structure i
// (M_i = s_i m_i, N_i = s_i n_i), the modified images of Eq.2 decompose exactly as
//   I_i~ = (I0~ + c0) + s_i/2 K_i~,  grad I_i~ = grad I0~ + s_i/2 grad K_i~,
//   T_i - I_i~ = (T0 - I0~) + s_i/2 (n_i (T0 + c0) - K_i~),
// so only the mask bits are stored, never the modified images.  Where neither mask of
// structure i touches the stencil, K_i~ = n_i = 0 and its terms reduce to
// lambda_i a0 d (numerator) and lambda_i a0^2 (denominator).
// ============================================================================
template <int KP, int TY>
__global__ void __launch_bounds__(kTileX *TY) k_force(ForceArgs a)
{
    constexpr int TXH = kTileX + 2, TYH = TY + 2, CELLS = TXH * TYH, NT = kTileX * TY;
    constexpr int KB_CELLS = KP > 0 ? CELLS : 1;
    __shared__ float W[3][KP + 1][CELLS];
    __shared__ uint8_t KB[3][KB_CELLS];
    __shared__ float red[NT / 64];

    const int tid = threadIdx.x;
    const int tx = tid % kTileX, ty = tid / kTileX;
    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, nxy = nx * ny;
    const int ntx = (nx + kTileX - 1) / kTileX;
    const int x0 = (blockIdx.x % ntx) * kTileX, y0 = (blockIdx.x / ntx) * TY;
    const int z0 = blockIdx.y * a.tz, z1 = min(z0 + a.tz, nz);

    const float *__restrict__ I0 = a.I0;
    const float *__restrict__ ux = a.u[0];
    const float *__restrict__ uy = a.u[1];
    const float *__restrict__ uz = a.u[2];

    // warped values of plane p (index clamped) into ring slot (p - z0 + 1) % 3
    auto plane = [&](int p) {
        const int pz = clampi(p, 0, nz - 1);
        const int s = (p - z0 + 1) % 3;
        for (int c = tid; c < CELLS; c += NT) {
            const int cy = c / TXH, cx = c - cy * TXH;
            const int gx = clampi(x0 - 1 + cx, 0, nx - 1);
            const int gy = clampi(y0 - 1 + cy, 0, ny - 1);
            const int v = gx + nx * gy + nxy * pz;
            const Split sx = split_axis(gx, ux[v], nx);
            const Split sy = split_axis(gy, uy[v], ny);
            const Split sz = split_axis(pz, uz[v], nz);
            const Corners q = corners(sx, sy, sz, nx, nxy);
            float f[8];
            f[0] = I0[q.r00 + q.x0];
            f[1] = I0[q.r00 + q.x1];
            f[2] = I0[q.r10 + q.x0];
            f[3] = I0[q.r10 + q.x1];
            f[4] = I0[q.r01 + q.x0];
            f[5] = I0[q.r01 + q.x1];
            f[6] = I0[q.r11 + q.x0];
            f[7] = I0[q.r11 + q.x1];
            W[s][0][c] = lerp8(f, q.tx, q.ty, q.tz);
            if constexpr (KP > 0) {
                const uint8_t *__restrict__ mb = a.mbits;
                uint32_t b[8];
                b[0] = mb[q.r00 + q.x0];
                b[1] = mb[q.r00 + q.x1];
                b[2] = mb[q.r10 + q.x0];
                b[3] = mb[q.r10 + q.x1];
                b[4] = mb[q.r01 + q.x0];
                b[5] = mb[q.r01 + q.x1];
                b[6] = mb[q.r11 + q.x0];
                b[7] = mb[q.r11 + q.x1];
                const uint32_t any = b[0] | b[1] | b[2] | b[3] | b[4] | b[5] | b[6] | b[7];
                KB[s][c] = (uint8_t)any;
                if (any) {
                    float g[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) g[j] = f[j] + a.c0;
#pragma unroll
                    for (int i = 0; i < KP; ++i) {
                        float kv = 0.f;
                        if ((any >> i) & 1u) {
                            float h[8];
#pragma unroll
                            for (int j = 0; j < 8; ++j) h[j] = ((b[j] >> i) & 1u) ? g[j] : 0.f;
                            kv = lerp8(h, q.tx, q.ty, q.tz);
                        }
                        W[s][1 + i][c] = kv;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < KP; ++i) W[s][1 + i][c] = 0.f;
                }
            }
        }
    };

    plane(z0 - 1);
    plane(z0);
    __syncthreads();

    float dacc = 0.f;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < nx && gy < ny;
    const int c = (ty + 1) * TXH + (tx + 1);
    for (int z = z0; z < z1; ++z) {
        plane(z + 1);
        __syncthreads();
        if (own) {
            const int v = gx + nx * gy + nxy * z;
            const int sm = (z - z0) % 3, s0 = (z - z0 + 1) % 3, sp = (z - z0 + 2) % 3;
            const float Ic = W[s0][0][c];
            const float g0x = 0.5f * (W[s0][0][c + 1] - W[s0][0][c - 1]);
            const float g0y = 0.5f * (W[s0][0][c + TXH] - W[s0][0][c - TXH]);
            const float g0z = 0.5f * (W[sp][0][c] - W[sm][0][c]);
            const float t0 = a.T0[v];
            const float d = t0 - Ic;
            const float a02 = __builtin_fmaf(g0z, g0z, __builtin_fmaf(g0y, g0y, g0x * g0x));
            float dx = 0.f, dy = 0.f, dz = 0.f;
            if (a02 != 0.f) {  // n = grad I0~ / |grad I0~| undefined at 0: no step
                const float a0 = sqrtf(a02);
                const float inv = 1.0f / a0;
                const float nxv = g0x * inv, nyv = g0y * inv, nzv = g0z * inv;
                float num = a0 * d;
                float den = __builtin_fmaf(d, d, a02);  // beta = d^2 (Thirion)
                if constexpr (KP > 0) {
                    const uint32_t tb = a.tbits[v];
                    const uint32_t kb = (uint32_t)KB[s0][c] | KB[s0][c - 1] | KB[s0][c + 1] |
                                        KB[s0][c - TXH] | KB[s0][c + TXH] | KB[sm][c] | KB[sp][c] | tb;
                    const float tc = t0 + a.c0;
                    float lam_off = 0.f;
#pragma unroll
                    for (int i = 0; i < KP; ++i) {
                        if (i < a.k) {
                            if ((kb >> i) & 1u) {
                                const float *Wi0 = W[s0][1 + i];
                                const float Kc = Wi0[c];
                                const float gkx = 0.5f * (Wi0[c + 1] - Wi0[c - 1]);
                                const float gky = 0.5f * (Wi0[c + TXH] - Wi0[c - TXH]);
                                const float gkz = 0.5f * (W[sp][1 + i][c] - W[sm][1 + i][c]);
                                const float proj =
                                    __builtin_fmaf(gkz, nzv, __builtin_fmaf(gky, nyv, gkx * nxv));
                                const float ai = __builtin_fmaf(a.hs[i], proj, a0);
                                const float ni = ((tb >> i) & 1u) ? tc : 0.f;
                                const float di = __builtin_fmaf(a.hs[i], ni - Kc, d);
                                const float la = a.lam[i] * ai;
                                num = __builtin_fmaf(la, di, num);
                                den = __builtin_fmaf(la, ai, den);
                            } else {
                                lam_off += a.lam[i];
                            }
                        }
                    }
                    num = __builtin_fmaf(lam_off * a0, d, num);
                    den = __builtin_fmaf(lam_off, a02, den);
                }
                const float vv = num / den;
                dx = vv * nxv;
                dy = vv * nyv;
                dz = vv * nzv;
            }
            a.du[0][v] = dx;
            a.du[1][v] = dy;
            a.du[2][v] = dz;
            if (a.partials != nullptr && a.uroi[v]) {
                const float e = d * a.inv_norm;
                dacc = __builtin_fmaf(e, e, dacc);
            }
        }
        __syncthreads();
    }

    if (a.partials != nullptr) {  // uniform over the launch
        dacc = wave_sum(dacc);
        if ((tid & 63) == 0) red[tid >> 6] = dacc;
        __syncthreads();
        if (tid == 0) {
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            a.partials[blockIdx.x + gridDim.x * blockIdx.y] = s;
        }
    }
}

// ============================================================================
// Separable Gaussian (kernel 1), sampled, radius R = ceil(3 sigma), normalised, clamped
// indices.  A block owns a 64 x TY column tile: each z plane (tile + R halo) is staged in
// LDS, filtered along x then y, and pushed into a register ring of 2R+1 planes that the
// z pass reads.  COMPOSE adds the composite update of kernel 4 on the smoothed step:
// out(x) = s(x) + u(x + s(x)) per component (u gathered trilinearly).
// ============================================================================
template <int R, int TY, bool COMPOSE>
__global__ void __launch_bounds__(kTileX *TY) k_smooth(SmoothArgs a)
{
    constexpr int WD = kTileX + 2 * R, HT = TY + 2 * R, NT = kTileX * TY;
    __shared__ float raw[3][HT][WD];
    __shared__ float xs[3][HT][kTileX];

    const int tid = threadIdx.x;
    const int tx = tid % kTileX, ty = tid / kTileX;
    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, nxy = nx * ny;
    const int ntx = (nx + kTileX - 1) / kTileX;
    const int x0 = (blockIdx.x % ntx) * kTileX, y0 = (blockIdx.x / ntx) * TY;
    const int z0 = blockIdx.y * a.tz, z1 = min(z0 + a.tz, nz);
    float w[R + 1];
#pragma unroll
    for (int m = 0; m <= R; ++m) w[m] = a.w[m];

    const float *__restrict__ in0 = a.in[0];
    const float *__restrict__ in1 = a.in[1];
    const float *__restrict__ in2 = a.in[2];

    auto plane = [&](int p, float out[3]) {
        const int pz = clampi(p, 0, nz - 1);
        for (int c = tid; c < HT * WD; c += NT) {
            const int r = c / WD, q = c - r * WD;
            const int gx = clampi(x0 - R + q, 0, nx - 1);
            const int gy = clampi(y0 - R + r, 0, ny - 1);
            const int v = gx + nx * gy + nxy * pz;
            raw[0][r][q] = in0[v];
            raw[1][r][q] = in1[v];
            raw[2][r][q] = in2[v];
        }
        __syncthreads();
        for (int c = tid; c < HT * kTileX; c += NT) {
            const int r = c / kTileX, q = c - r * kTileX;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float s = w[0] * raw[k][r][q + R];
#pragma unroll
                for (int m = 1; m <= R; ++m) s = __builtin_fmaf(w[m], raw[k][r][q + R - m] + raw[k][r][q + R + m], s);
                xs[k][r][q] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = w[0] * xs[k][ty + R][tx];
#pragma unroll
            for (int m = 1; m <= R; ++m) s = __builtin_fmaf(w[m], xs[k][ty + R - m][tx] + xs[k][ty + R + m][tx], s);
            out[k] = s;
        }
    };

    float ring[3][2 * R + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m <= 2 * R; ++m) ring[k][m] = 0.f;
    auto push = [&](const float v3[3]) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int m = 0; m < 2 * R; ++m) ring[k][m] = ring[k][m + 1];
            ring[k][2 * R] = v3[k];
        }
    };

    float v3[3];
    for (int q = 0; q < 2 * R; ++q) {
        plane(z0 - R + q, v3);
        push(v3);
    }
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < nx && gy < ny;
    for (int z = z0; z < z1; ++z) {
        plane(z + R, v3);
        push(v3);
        if (own) {
            const int v = gx + nx * gy + nxy * z;
            float s[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float t = w[0] * ring[k][R];
#pragma unroll
                for (int m = 1; m <= R; ++m) t = __builtin_fmaf(w[m], ring[k][R - m] + ring[k][R + m], t);
                s[k] = t;
            }
            if constexpr (COMPOSE) {
                const Split sx = split_axis(gx, s[0], nx);
                const Split sy = split_axis(gy, s[1], ny);
                const Split sz = split_axis(z, s[2], nz);
                const Corners q = corners(sx, sy, sz, nx, nxy);
#pragma unroll
                for (int k = 0; k < 3; ++k) a.out[k][v] = s[k] + trilinear(a.u[k], q);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) a.out[k][v] = s[k];
            }
        }
    }
}

// ============================================================================
// Stopping metric: delta = sqrt(sum of the per-block partials / |UROI|), summed in a fixed
// order in double precision (kernel 5).
// ============================================================================
__global__ void __launch_bounds__(256) k_delta_finalize(const float *partials, int nblocks,
                                                        const int64_t *count, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += 256) s += (double)partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t n = *count;
        out[0] = n > 0 ? sqrt(red[0] / (double)n) : 0.0;
    }
}

// ============================================================================
// Pyramid.  Restriction R(F)(j) = (G_sigma * F)(2j) as three 1D passes that each keep the
// even samples along their axis; prolongation u_f(x) = 2 u_c(x / 2).
// ============================================================================
struct Taps {
    float w[kMaxRadius + 1];
};

__global__ void __launch_bounds__(256) k_restrict_pass(const float *__restrict__ in,
                                                       float *__restrict__ out, Dims din,
                                                       Dims dout, int axis, Taps t, int R)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= dout.n()) return;
    const int ox = (int)(idx % dout.nx);
    const int oy = (int)((idx / dout.nx) % dout.ny);
    const int oz = (int)(idx / ((int64_t)dout.nx * dout.ny));
    const int ext = axis == 0 ? din.nx : (axis == 1 ? din.ny : din.nz);
    const int ctr = 2 * (axis == 0 ? ox : (axis == 1 ? oy : oz));
    auto at = [&](int m) {
        const int q = clampi(ctr + m, 0, ext - 1);
        const int ix = axis == 0 ? q : ox, iy = axis == 1 ? q : oy, iz = axis == 2 ? q : oz;
        return in[ix + (int64_t)din.nx * (iy + (int64_t)din.ny * iz)];
    };
    float s = t.w[0] * at(0);
    for (int m = 1; m <= R; ++m) s = __builtin_fmaf(t.w[m], at(-m) + at(m), s);
    out[idx] = s;
}

struct Field3 {
    const float *p[3];
};
struct Field3W {
    float *p[3];
};

__global__ void __launch_bounds__(256) k_prolong(Field3 uc, Dims dc, Field3W uf, Dims df)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= df.n()) return;
    const int i = (int)(idx % df.nx);
    const int j = (int)((idx / df.nx) % df.ny);
    const int l = (int)(idx / ((int64_t)df.nx * df.ny));
    auto half = [](int f, int n) {  // coarse position f / 2, clamped to [0, n - 1]
        Split s;
        s.i0 = f >> 1;
        s.t = (f & 1) ? 0.5f : 0.f;
        if (s.i0 >= n - 1) {
            s.i0 = n - 1;
            s.t = 0.f;
        }
        s.i1 = min(s.i0 + 1, n - 1);
        return s;
    };
    const Corners q = corners(half(i, dc.nx), half(j, dc.ny), half(l, dc.nz), dc.nx, dc.nx * dc.ny);
#pragma unroll
    for (int k = 0; k < 3; ++k) uf.p[k][idx] = 2.0f * trilinear(uc.p[k], q);
}

// ============================================================================
// Masks and the UROI (section 2.2)
// ============================================================================
struct MaskPtrs {
    const uint8_t *p[kMaxStructs];
};

__global__ void __launch_bounds__(256) k_pack_masks(MaskPtrs m, int k, int64_t n, uint8_t *bits)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t b = 0;
    for (int i = 0; i < k; ++i)
        if (m.p[i][v]) b |= 1u << i;
    bits[v] = (uint8_t)b;
}

// distance along x to the nearest voxel whose bits intersect `sel`, capped at 255
__global__ void __launch_bounds__(256) k_rowdist(const uint8_t *__restrict__ bits, uint8_t sel,
                                                 Dims d, uint8_t *__restrict__ dist)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= (int64_t)d.ny * d.nz) return;
    const uint8_t *b = bits + row * d.nx;
    uint8_t *o = dist + row * d.nx;
    int last = -100000;
    for (int i = 0; i < d.nx; ++i) {
        if (b[i] & sel) last = i;
        o[i] = (uint8_t)min(i - last, 255);
    }
    int next = 100000;
    for (int i = d.nx - 1; i >= 0; --i) {
        if (b[i] & sel) next = i;
        o[i] = (uint8_t)min((int)o[i], min(next - i, 255));
    }
}

// half-widths along x of the ellipsoidal element for every (dy, dz); -1 = empty row
struct Element {
    int8_t w[2 * kMaxUroiMargin + 1][2 * kMaxUroiMargin + 1];
    int ry, rz;
};

__global__ void __launch_bounds__(256) k_dilate(const uint8_t *__restrict__ dist, Dims d, Element e,
                                                uint8_t *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.n()) return;
    const int i = (int)(idx % d.nx);
    const int j = (int)((idx / d.nx) % d.ny);
    const int l = (int)(idx / ((int64_t)d.nx * d.ny));
    uint8_t in = 0;
    for (int c = -e.rz; c <= e.rz && !in; ++c) {
        const int ll = l + c;
        if (ll < 0 || ll >= d.nz) continue;
        for (int b = -e.ry; b <= e.ry; ++b) {
            const int jj = j + b;
            const int w = e.w[c + kMaxUroiMargin][b + kMaxUroiMargin];
            if (w < 0 || jj < 0 || jj >= d.ny) continue;
            if ((int)dist[i + (int64_t)d.nx * (jj + (int64_t)d.ny * ll)] <= w) {
                in = 1;
                break;
            }
        }
    }
    out[idx] = in;
}

__global__ void __launch_bounds__(256) k_count_partials(const uint8_t *__restrict__ m, int64_t n,
                                                        uint8_t sel, int64_t *partials)
{
    __shared__ int64_t red[256];
    int64_t s = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256)
        s += (m[v] & sel) ? 1 : 0;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_i64(const int64_t *partials, int n, int64_t *out)
{
    __shared__ int64_t red[256];
    int64_t s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// sums of T0 and counts inside structure `bit` and in its shell (dilated minus itself)
__global__ void __launch_bounds__(256) k_sign_partials(const float *__restrict__ T0,
                                                       const uint8_t *__restrict__ tbits,
                                                       const uint8_t *__restrict__ dil, uint8_t sel,
                                                       int64_t n, double *partials)
{
    __shared__ double red[4][256];
    double si = 0, ci = 0, so = 0, co = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        if (tbits[v] & sel) {
            si += T0[v];
            ci += 1.0;
        } else if (dil[v]) {
            so += T0[v];
            co += 1.0;
        }
    }
    red[0][threadIdx.x] = si;
    red[1][threadIdx.x] = ci;
    red[2][threadIdx.x] = so;
    red[3][threadIdx.x] = co;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) partials[4 * blockIdx.x + q] = red[q][0];
}

__global__ void __launch_bounds__(64) k_sum_f64x4(const double *partials, int n, double *out)
{
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partials[4 * i + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ============================================================================
// Public warp (kernel 4 on images and masks)
// ============================================================================
__global__ void __launch_bounds__(256) k_warp_linear(const float *__restrict__ src, Dims d, Field3 u,
                                                     float *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.n()) return;
    const int i = (int)(idx % d.nx);
    const int j = (int)((idx / d.nx) % d.ny);
    const int l = (int)(idx / ((int64_t)d.nx * d.ny));
    const Corners q = corners(split_axis(i, u.p[0][idx], d.nx), split_axis(j, u.p[1][idx], d.ny),
                              split_axis(l, u.p[2][idx], d.nz), d.nx, d.nx * d.ny);
    out[idx] = trilinear(src, q);
}

__global__ void __launch_bounds__(256) k_warp_mask(const uint8_t *__restrict__ src, Dims d, Field3 u,
                                                   uint8_t *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.n()) return;
    const int i = (int)(idx % d.nx);
    const int j = (int)((idx / d.nx) % d.ny);
    const int l = (int)(idx / ((int64_t)d.nx * d.ny));
    const Corners q = corners(split_axis(i, u.p[0][idx], d.nx), split_axis(j, u.p[1][idx], d.ny),
                              split_axis(l, u.p[2][idx], d.nz), d.nx, d.nx * d.ny);
    float v[8];
    v[0] = src[q.r00 + q.x0] ? 1.f : 0.f;
    v[1] = src[q.r00 + q.x1] ? 1.f : 0.f;
    v[2] = src[q.r10 + q.x0] ? 1.f : 0.f;
    v[3] = src[q.r10 + q.x1] ? 1.f : 0.f;
    v[4] = src[q.r01 + q.x0] ? 1.f : 0.f;
    v[5] = src[q.r01 + q.x1] ? 1.f : 0.f;
    v[6] = src[q.r11 + q.x0] ? 1.f : 0.f;
    v[7] = src[q.r11 + q.x1] ? 1.f : 0.f;
    out[idx] = lerp8(v, q.tx, q.ty, q.tz) >= 0.5f ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_fill(float *p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

__global__ void __launch_bounds__(256) k_nonfinite(const float *__restrict__ p, int64_t n, int *flag)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        bad |= !isfinite(p[i]);
    if (bad) *flag = 1;  // every writer stores the same value
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ----------------------------------------------------------------------------- launchers

static int tiles_xy(Dims d, int ty) { return ((d.nx + kTileX - 1) / kTileX) * ((d.ny + ty - 1) / ty); }

int force_partial_blocks(Dims d, int ty, int tz) { return tiles_xy(d, ty) * ((d.nz + tz - 1) / tz); }

template <int KP, int TY>
static hipError_t force_kp_ty(const ForceArgs &a, hipStream_t s)
{
    dim3 grid(tiles_xy(a.d, TY), (a.d.nz + a.tz - 1) / a.tz);
    hipLaunchKernelGGL((k_force<KP, TY>), grid, dim3(kTileX * TY), 0, s, a);
    return hipGetLastError();
}

template <int TY>
static hipError_t force_ty(const ForceArgs &a, int kp, hipStream_t s)
{
    switch (kp) {
    case 0: return force_kp_ty<0, TY>(a, s);
    case 1: return force_kp_ty<1, TY>(a, s);
    case 2: return force_kp_ty<2, TY>(a, s);
    case 4: return force_kp_ty<4, TY>(a, s);
    case 8: return force_kp_ty<8, TY>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_force(const ForceArgs &a, int kp, int ty, hipStream_t s, int *blocks_out)
{
    if (blocks_out) *blocks_out = force_partial_blocks(a.d, ty, a.tz);
    switch (ty) {
    case 4: return force_ty<4>(a, kp, s);
    case 8: return force_ty<8>(a, kp, s);
    default: return hipErrorInvalidValue;
    }
}

template <int R, int TY>
static hipError_t smooth_r_ty(const SmoothArgs &a, bool compose, hipStream_t s)
{
    dim3 grid(tiles_xy(a.d, TY), (a.d.nz + a.tz - 1) / a.tz);
    if (compose)
        hipLaunchKernelGGL((k_smooth<R, TY, true>), grid, dim3(kTileX * TY), 0, s, a);
    else
        hipLaunchKernelGGL((k_smooth<R, TY, false>), grid, dim3(kTileX * TY), 0, s, a);
    return hipGetLastError();
}

template <int TY>
static hipError_t smooth_ty(const SmoothArgs &a, int radius, bool compose, hipStream_t s)
{
    switch (radius) {
    case 0: return smooth_r_ty<0, TY>(a, compose, s);
    case 1: return smooth_r_ty<1, TY>(a, compose, s);
    case 2: return smooth_r_ty<2, TY>(a, compose, s);
    case 3: return smooth_r_ty<3, TY>(a, compose, s);
    case 4: return smooth_r_ty<4, TY>(a, compose, s);
    case 5: return smooth_r_ty<5, TY>(a, compose, s);
    case 6: return smooth_r_ty<6, TY>(a, compose, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_smooth(const SmoothArgs &a, int radius, bool compose, int ty, hipStream_t s)
{
    switch (ty) {
    case 4: return smooth_ty<4>(a, radius, compose, s);
    case 8: return smooth_ty<8>(a, radius, compose, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_delta_finalize(const float *partials, int nblocks, const int64_t *count, double *out,
                                 float, hipStream_t s)
{
    hipLaunchKernelGGL(k_delta_finalize, dim3(1), dim3(256), 0, s, partials, nblocks, count, out);
    return hipGetLastError();
}

hipError_t launch_restrict_pass(const float *in, float *out, Dims din, int axis, const float *w, int radius,
                                hipStream_t s)
{
    if (radius < 0 || radius > kMaxRadius || axis < 0 || axis > 2) return hipErrorInvalidValue;
    Dims dout = din;
    if (axis == 0) dout.nx = (din.nx + 1) / 2;
    if (axis == 1) dout.ny = (din.ny + 1) / 2;
    if (axis == 2) dout.nz = (din.nz + 1) / 2;
    Taps t{};
    for (int m = 0; m <= radius; ++m) t.w[m] = w[m];
    hipLaunchKernelGGL(k_restrict_pass, dim3(blocks_for(dout.n(), 256)), dim3(256), 0, s, in, out, din, dout,
                       axis, t, radius);
    return hipGetLastError();
}

hipError_t launch_prolong(const float *const uc[3], Dims dc, float *const uf[3], Dims df, hipStream_t s)
{
    Field3 c{{uc[0], uc[1], uc[2]}};
    Field3W f{{uf[0], uf[1], uf[2]}};
    hipLaunchKernelGGL(k_prolong, dim3(blocks_for(df.n(), 256)), dim3(256), 0, s, c, dc, f, df);
    return hipGetLastError();
}

hipError_t launch_pack_masks(const uint8_t *const *planes, int k, int64_t n, uint8_t *bits, hipStream_t s)
{
    if (k < 0 || k > kMaxStructs) return hipErrorInvalidValue;
    MaskPtrs m{};
    for (int i = 0; i < k; ++i) m.p[i] = planes[i];
    hipLaunchKernelGGL(k_pack_masks, dim3(blocks_for(n, 256)), dim3(256), 0, s, m, k, n, bits);
    return hipGetLastError();
}

// ellipsoid half-widths, decided in double exactly as the membership test
// (a/rx)^2 + (b/ry)^2 + (c/rz)^2 <= 1 of the element
static Element make_element(const int r[3])
{
    Element e{};
    e.ry = r[1];
    e.rz = r[2];
    for (int c = -kMaxUroiMargin; c <= kMaxUroiMargin; ++c)
        for (int b = -kMaxUroiMargin; b <= kMaxUroiMargin; ++b) {
            int best = -1;
            if (c >= -r[2] && c <= r[2] && b >= -r[1] && b <= r[1])
                for (int a = 0; a <= r[0]; ++a) {
                    double q = 0.0;
                    if (r[0] > 0) q += (double)(a * a) / (double)(r[0] * r[0]);
                    if (r[1] > 0) q += (double)(b * b) / (double)(r[1] * r[1]);
                    if (r[2] > 0) q += (double)(c * c) / (double)(r[2] * r[2]);
                    if (q <= 1.0) best = a;
                }
            e.w[c + kMaxUroiMargin][b + kMaxUroiMargin] = (int8_t)best;
        }
    return e;
}

static hipError_t dilate_sel(const uint8_t *bits, uint8_t sel, Dims d, const int margin[3], uint8_t *rowdist,
                             uint8_t *out, hipStream_t s)
{
    for (int a = 0; a < 3; ++a)
        if (margin[a] < 0 || margin[a] > kMaxUroiMargin) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rowdist, dim3(blocks_for((int64_t)d.ny * d.nz, 256)), dim3(256), 0, s, bits, sel, d,
                       rowdist);
    Element e = make_element(margin);
    hipLaunchKernelGGL(k_dilate, dim3(blocks_for(d.n(), 256)), dim3(256), 0, s, rowdist, d, e, out);
    return hipGetLastError();
}

hipError_t launch_uroi(const uint8_t *tbits, Dims d, const int margin[3], uint8_t *rowdist, uint8_t *uroi,
                       hipStream_t s)
{
    return dilate_sel(tbits, 0xFF, d, margin, rowdist, uroi, s);
}

hipError_t launch_dilate_bit(const uint8_t *bits, int bit, Dims d, const int margin[3], uint8_t *rowdist,
                             uint8_t *out, hipStream_t s)
{
    return dilate_sel(bits, (uint8_t)(1u << bit), d, margin, rowdist, out, s);
}

hipError_t launch_count(const uint8_t *m, int64_t n, uint8_t bitmask, int64_t *partials, int *nparts,
                        int64_t *out, hipStream_t s)
{
    const int G = 256;
    if (nparts) *nparts = G;
    hipLaunchKernelGGL(k_count_partials, dim3(G), dim3(256), 0, s, m, n, bitmask, partials);
    hipLaunchKernelGGL(k_sum_i64, dim3(1), dim3(256), 0, s, partials, G, out);
    return hipGetLastError();
}

hipError_t launch_sign_stats(const float *T0, const uint8_t *tbits, const uint8_t *dil, int bit, int64_t n,
                             double *partials, int *nparts, double *out4, hipStream_t s)
{
    const int G = 128;
    if (nparts) *nparts = G;
    hipLaunchKernelGGL(k_sign_partials, dim3(G), dim3(256), 0, s, T0, tbits, dil, (uint8_t)(1u << bit), n,
                       partials);
    hipLaunchKernelGGL(k_sum_f64x4, dim3(1), dim3(64), 0, s, partials, G, out4);
    return hipGetLastError();
}

hipError_t launch_warp_linear(const float *src, Dims d, const float *const u[3], float *out, hipStream_t s)
{
    Field3 f{{u[0], u[1], u[2]}};
    hipLaunchKernelGGL(k_warp_linear, dim3(blocks_for(d.n(), 256)), dim3(256), 0, s, src, d, f, out);
    return hipGetLastError();
}

hipError_t launch_warp_mask(const uint8_t *src, Dims d, const float *const u[3], uint8_t *out, hipStream_t s)
{
    Field3 f{{u[0], u[1], u[2]}};
    hipLaunchKernelGGL(k_warp_mask, dim3(blocks_for(d.n(), 256)), dim3(256), 0, s, src, d, f, out);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s)
{
    const unsigned g = (unsigned)std::min<int64_t>(blocks_for(n, 256), 4096);
    hipLaunchKernelGGL(k_fill, dim3(g > 0 ? g : 1), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const float *p, int64_t n, int *flag, hipStream_t s)
{
    const unsigned g = (unsigned)std::min<int64_t>(blocks_for(n, 256), 2048);
    hipLaunchKernelGGL(k_nonfinite, dim3(g > 0 ? g : 1), dim3(256), 0, s, p, n, flag);
    return hipGetLastError();
}

}  // namespace cgdir
