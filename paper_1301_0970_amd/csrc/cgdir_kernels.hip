// HIP kernels of libcgdir for gfx950 (MI355X): the per-voxel CG-DIR iteration
// (section 2.1, Eqs. 5-7; section 2.2, the five data-parallel kernels) and its
// pyramid / mask / metric helpers.  FP32 arithmetic, x-fastest volumes, SoA fields.
//
// Every per-voxel result depends only on the voxel and the data, never on the tile
// shape or on what else shares the launch, so results are bitwise reproducible
// whether a pair runs alone or batched.
#include <math.h>

#include <type_traits>

#include "cgdir_internal.h"

namespace cgdir {
namespace {

__device__ __forceinline__ float lerpf(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Loads and stores at an element index.  A volume holds at most 2^30 voxels, so a byte
// offset fits in 32 bits and the address is a scalar base plus a 32-bit vector offset: no
// 64-bit address arithmetic per access.
template <class T>
__device__ __forceinline__ T ldg(const T *base, uint32_t i)
{
    return *(const T *)((const char *)base + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stg(T *base, uint32_t i, T v)
{
    *(T *)((char *)base + i * (uint32_t)sizeof(T)) = v;
}

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
    const float pb = (float)i + fu;
    const float top = (float)(n - 1);
    // below 0 or at/after the last voxel: the border voxel with weight 0; NaN keeps an
    // in-bounds index (max/min return the non-NaN operand) and a NaN weight.  Branch free.
    const bool outside = pb < 0.f || pb >= top;
    Split s;
    s.i0 = (int)fminf(fmaxf(pb, 0.f), top);
    s.i1 = min(s.i0 + 1, n - 1);
    s.t = outside ? 0.f : u - fu;
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
    v[0] = ldg(f, c.r00 + c.x0);
    v[1] = ldg(f, c.r00 + c.x1);
    v[2] = ldg(f, c.r10 + c.x0);
    v[3] = ldg(f, c.r10 + c.x1);
    v[4] = ldg(f, c.r01 + c.x0);
    v[5] = ldg(f, c.r01 + c.x1);
    v[6] = ldg(f, c.r11 + c.x0);
    v[7] = ldg(f, c.r11 + c.x1);
    return lerp8(v, c.tx, c.ty, c.tz);
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

struct Field3 {
    const float *p[3];
};
struct Field3W {
    float *p[3];
};

// XCD-aware block order.  The dispatcher hands consecutive block ids to the 8 XCDs in
// turn; the blocks one XCD receives are mapped onto a contiguous range of logical tiles, so
// that tiles sharing halo cache lines run on the same L2.  Logical order: x tile fastest,
// then y tile, then z chunk, so that the blocks an XCD runs at one time cover a compact
// patch of neighbouring columns marching through z together.  Bijective on [0, total).
__device__ __forceinline__ int xcd_logical(int b, int total)
{
    const int per = total >> 3, rem = total & 7;
    const int x = b & 7, local = b >> 3;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + local;
}

struct TileCoord {
    int x0, y0, z0, z1;
};

// logical tile L of a volume: x tile fastest, then y tile, then z chunk
__device__ __forceinline__ TileCoord tile_of(int ty_rows, int tz, const Dims &d, int L)
{
    const int ntx = (d.nx + kTileX - 1) / kTileX;
    const int nty = (d.ny + ty_rows - 1) / ty_rows;
    const int tx = L % ntx, t = L / ntx;
    TileCoord c;
    c.x0 = tx * kTileX;
    c.y0 = (t % nty) * ty_rows;
    c.z0 = (t / nty) * tz;
    c.z1 = min(c.z0 + tz, d.nz);
    return c;
}

// Warp of the masked moving image m_i (I0 + c0) at voxel (px, py, pz) with the field u:
// K_i~ of the decomposition below, for the structures selected by `bit`.
__device__ __forceinline__ float warp_masked(const StepArgs &a, int px, int py, int pz, uint32_t bit)
{
    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, nxy = nx * ny;
    const int v = px + nx * py + nxy * pz;
    const Corners q = corners(split_axis(px, ldg(a.u[0], v), nx), split_axis(py, ldg(a.u[1], v), ny),
                              split_axis(pz, ldg(a.u[2], v), nz), nx, nxy);
    const int o[8] = {q.r00 + q.x0, q.r00 + q.x1, q.r10 + q.x0, q.r10 + q.x1,
                      q.r01 + q.x0, q.r01 + q.x1, q.r11 + q.x0, q.r11 + q.x1};
    float h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = (ldg(a.mbits, o[j]) & bit) ? ldg(a.I0, o[j]) + a.c0 : 0.f;
    return lerp8(h, q.tx, q.ty, q.tz);
}

// ============================================================================
// Warp of the moving image (kernel 4), split into issue (positions, gathers in flight)
// and finish (interpolation, mask bits, stores) so that callers can overlap the gathers
// with other work.  The moving-mask bits are read only where the brick occupancy map says
// a structure is near.
// ============================================================================
struct WarpPending {
    float g[8];
    float t[3];
    int b[3];
    uint32_t occ;
};

__device__ __forceinline__ void warp_issue(const WarpArgs &w, int gx, int gy, int gz, float ux, float uy, float uz,
                                           WarpPending &p)
{
    const int nx = w.d.nx, ny = w.d.ny, nz = w.d.nz, nxy = nx * ny;
    const Split sx = split_axis(gx, ux, nx), sy = split_axis(gy, uy, ny), sz = split_axis(gz, uz, nz);
    const Corners q = corners(sx, sy, sz, nx, nxy);
    const float *__restrict__ I0 = w.I0;
    p.g[0] = ldg(I0, q.r00 + q.x0);
    p.g[1] = ldg(I0, q.r00 + q.x1);
    p.g[2] = ldg(I0, q.r10 + q.x0);
    p.g[3] = ldg(I0, q.r10 + q.x1);
    p.g[4] = ldg(I0, q.r01 + q.x0);
    p.g[5] = ldg(I0, q.r01 + q.x1);
    p.g[6] = ldg(I0, q.r11 + q.x0);
    p.g[7] = ldg(I0, q.r11 + q.x1);
    p.t[0] = q.tx;
    p.t[1] = q.ty;
    p.t[2] = q.tz;
    p.b[0] = sx.i0;
    p.b[1] = sy.i0;
    p.b[2] = sz.i0;
    p.occ = w.mbits != nullptr ? ldg(w.mocc, (sx.i0 >> 3) + w.bnx * ((sy.i0 >> 3) + w.bny * (sz.i0 >> 3))) : 0u;
}

__device__ __forceinline__ void warp_finish(const WarpArgs &w, const WarpPending &p, int v)
{
    stg(w.wI0, v, lerp8(p.g, p.t[0], p.t[1], p.t[2]));
    if (w.mbits == nullptr) return;
    uint32_t any = 0;
    if (p.occ) {  // a structure is near: mask bits at the 8 corners
        const int nx = w.d.nx, ny = w.d.ny, nz = w.d.nz, nxy = nx * ny;
        const int i0 = p.b[0], j0 = p.b[1], l0 = p.b[2];
        const int i1 = min(i0 + 1, nx - 1), j1 = min(j0 + 1, ny - 1), l1 = min(l0 + 1, nz - 1);
        const uint8_t *__restrict__ mb = w.mbits;
        uint32_t b[8];
        b[0] = ldg(mb, i0 + nx * j0 + nxy * l0);
        b[1] = ldg(mb, i1 + nx * j0 + nxy * l0);
        b[2] = ldg(mb, i0 + nx * j1 + nxy * l0);
        b[3] = ldg(mb, i1 + nx * j1 + nxy * l0);
        b[4] = ldg(mb, i0 + nx * j0 + nxy * l1);
        b[5] = ldg(mb, i1 + nx * j0 + nxy * l1);
        b[6] = ldg(mb, i0 + nx * j1 + nxy * l1);
        b[7] = ldg(mb, i1 + nx * j1 + nxy * l1);
        any = b[0] | b[1] | b[2] | b[3] | b[4] | b[5] | b[6] | b[7];
        if (any != 0 && (any & (any - 1)) == 0) {  // one structure: its K_i~ here
            float h[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) h[m] = (b[m] & any) ? p.g[m] + w.c0 : 0.f;
            stg(w.K, v, lerp8(h, p.t[0], p.t[1], p.t[2]));
        }
    }
    stg(w.F, v, (uint8_t)any);
}

// ============================================================================
// Eq.7 at one voxel (kernels 2 and 3 on the warped moving image).
//
// With s_i the sign of structure i (M_i = s_i m_i, N_i = s_i n_i), the modified images of
// Eq.2 decompose exactly (trilinear interpolation and central differences are linear):
//   I_i~ = (I0~ + c0) + s_i/2 K_i~,   grad I_i~ = grad I0~ + s_i/2 grad K_i~,
//   T_i - I_i~ = (T0 - I0~) + s_i/2 (n_i (T0 + c0) - K_i~),   K_i~ = (m_i (I0 + c0)) o (Id + u).
// Where neither mask of structure i touches the stencil, K_i~ = n_i = 0 and its terms of
// Eq.7 reduce to lambda_i a0 d (numerator) and lambda_i a0^2 (denominator): that is the
// whole computation for most voxels.  Where one structure touches it, K_i~ at the stencil
// cells comes from the warp; where several do, K_i~ is re-evaluated from the field.
//
// w: I0~ at the voxel and its six clamped neighbours (centre, -x, +x, -y, +y, -z, +z);
// f: their stencil structure bits (zero when the level has no contour terms);
// lamt: lambda_i at [i] and the sum of the other weights in index order at [kMaxStructs + i];
// kl, ks: K~ staged in LDS: the centre of plane slot s at kl[ks[s]] (s: 0 this plane, 1 the
// one below, 2 the one above; rows kRow apart), read only where f[q] is nonzero; without
// staging (kLds false) K~ is read from memory.
// ============================================================================
// kAniso: the voxel sizes along x and y differ (else the y axis takes x's scale).
template <bool kLds, int kRow, bool kAniso>
__device__ __forceinline__ void force_at(const StepArgs &a, const float w[7], const uint32_t f[7], float t0,
                                         uint32_t tb, int gx, int gy, int gz, const float *lamt, const float *kl,
                                         const int ks[3], float du[3], float *dout)
{
    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, nxy = nx * ny;
    // central differences of I0~ (times 2 h: the gradient is gs times these)
    const float ex = w[2] - w[1], ey = w[4] - w[3], ez = w[6] - w[5];
    const float d = t0 - w[0];
    *dout = d;
    // (a pair with square in-plane voxels takes the same arithmetic in both instantiations, so
    // that its result does not depend on the other pairs of its launch)
    const float a02 = kAniso && a.gs2[0] != a.gs2[1]
                          ? __builtin_fmaf(a.gs2[2], ez * ez, __builtin_fmaf(a.gs2[1], ey * ey, a.gs2[0] * (ex * ex)))
                          : __builtin_fmaf(a.gs2[2], ez * ez, a.gs2[0] * __builtin_fmaf(ey, ey, ex * ex));
    const float sy = kAniso ? a.gs[1] : a.gs[0];  // the y scale
    du[0] = du[1] = du[2] = 0.f;
    // n = grad I0~ / |grad I0~| undefined at 0: no step (also below the smallest normal
    // float, where the step is below 1e-19 voxel; NaN goes on and is reported)
    if (a02 < 1.17549435e-38f) return;
    const uint32_t kb = f[0] | f[1] | f[2] | f[3] | f[4] | f[5] | f[6] | tb;
    if (kb == 0) {
        // no structure touches the stencil: every contour term of Eq.7 reduces to lambda_i a0 d
        // (numerator) and lambda_i a0^2 (denominator), so v n = L a0 d n / (L a0^2 + d^2) with
        // L = 1 + sum lambda_i, which is L d grad I0~ / (L a0^2 + d^2): the unit vector n is
        // never formed.  In voxels along each axis the step is that times 2 gs, i.e. 2 gs^2 L d
        // e / (L a0^2 + d^2) for the difference e (beta = d^2, Thirion).
        const float q = d * __builtin_amdgcn_rcpf(__builtin_fmaf(a.far_l1, a02, d * d));  // ~1 ulp
        du[0] = (a.far_c[0] * q) * ex;
        du[1] = ((kAniso ? a.far_c[1] : a.far_c[0]) * q) * ey;
        du[2] = (a.far_c[2] * q) * ez;
        return;
    }
    const float g0x = a.gs[0] * ex, g0y = sy * ey, g0z = a.gs[2] * ez;
    const float inv = __builtin_amdgcn_rsqf(a02);  // hardware 1/sqrt, ~1 ulp
    const float a0 = a02 * inv;
    const float nxv = g0x * inv, nyv = g0y * inv, nzv = g0z * inv;
    float num = a0 * d;
    float den = __builtin_fmaf(d, d, a02);  // beta = d^2 (Thirion)
    float lam_off;
    {
        const int xm = max(gx - 1, 0), xp = min(gx + 1, nx - 1);
        const int ym = max(gy - 1, 0), yp = min(gy + 1, ny - 1);
        const int zm = max(gz - 1, 0), zp = min(gz + 1, nz - 1);
        if ((kb & (kb - 1)) == 0) {
            // one structure i near: K_i~ at each stencil cell from the warp (0 where the
            // cell's corners miss the structure)
            const int i = __builtin_ctz(kb);
            float Kq[7];
            if constexpr (kLds) {
                // (read unconditionally, then selected: the ring cells of the stencil always
                // lie in the block's LDS, and a stale value is never selected)
                const float *k0 = kl + ks[0];
                const float kv[7] = {k0[0], k0[-1], k0[1], k0[-kRow], k0[kRow], kl[ks[1]], kl[ks[2]]};
#pragma unroll
                for (int q = 0; q < 7; ++q) Kq[q] = f[q] ? kv[q] : 0.f;
            } else {
                const float *__restrict__ K = a.K;
                const int v = gx + nx * gy + nxy * gz;
                Kq[0] = f[0] ? ldg(K, v) : 0.f;
                Kq[1] = f[1] ? ldg(K, xm + nx * gy + nxy * gz) : 0.f;
                Kq[2] = f[2] ? ldg(K, xp + nx * gy + nxy * gz) : 0.f;
                Kq[3] = f[3] ? ldg(K, gx + nx * ym + nxy * gz) : 0.f;
                Kq[4] = f[4] ? ldg(K, gx + nx * yp + nxy * gz) : 0.f;
                Kq[5] = f[5] ? ldg(K, gx + nx * gy + nxy * zm) : 0.f;
                Kq[6] = f[6] ? ldg(K, gx + nx * gy + nxy * zp) : 0.f;
            }
            const float Kc = Kq[0];
            const float gkx = a.gs[0] * (Kq[2] - Kq[1]);
            const float gky = sy * (Kq[4] - Kq[3]);
            const float gkz = a.gs[2] * (Kq[6] - Kq[5]);
            const float proj = __builtin_fmaf(gkz, nzv, __builtin_fmaf(gky, nyv, gkx * nxv));
            const float hs = ((a.neg >> i) & 1u) ? -0.5f : 0.5f;
            const float ai = __builtin_fmaf(hs, proj, a0);
            const float ni = (tb & kb) ? t0 + a.c0 : 0.f;
            const float di = __builtin_fmaf(hs, ni - Kc, d);
            const float la = lamt[i] * ai;
            lam_off = lamt[kMaxStructs + i];
            num = __builtin_fmaf(la, di, num);
            den = __builtin_fmaf(la, ai, den);
        } else {  // several structures near: their terms in full
            lam_off = 0.f;
            const float tc0 = t0 + a.c0;
#pragma unroll 1
            for (int i = 0; i < a.k; ++i) {
                const uint32_t bit = 1u << i;
                if (kb & bit) {
                    // K_i~ at the centre and the six clamped neighbours (+x, -x, +y, -y, +z, -z)
                    float Kq[7];
#pragma unroll 1
                    for (int q = 0; q < 7; ++q) {
                        const int px = q == 1 ? xp : (q == 2 ? xm : gx);
                        const int py = q == 3 ? yp : (q == 4 ? ym : gy);
                        const int pz = q == 5 ? zp : (q == 6 ? zm : gz);
                        Kq[q] = warp_masked(a, px, py, pz, bit);
                    }
                    const float Kc = Kq[0];
                    const float gkx = a.gs[0] * (Kq[1] - Kq[2]);
                    const float gky = sy * (Kq[3] - Kq[4]);
                    const float gkz = a.gs[2] * (Kq[5] - Kq[6]);
                    const float proj = __builtin_fmaf(gkz, nzv, __builtin_fmaf(gky, nyv, gkx * nxv));
                    const float hs = ((a.neg >> i) & 1u) ? -0.5f : 0.5f;
                    const float ai = __builtin_fmaf(hs, proj, a0);
                    const float ni = (tb & bit) ? tc0 : 0.f;
                    const float di = __builtin_fmaf(hs, ni - Kc, d);
                    const float la = a.lam[i] * ai;
                    num = __builtin_fmaf(la, di, num);
                    den = __builtin_fmaf(la, ai, den);
                } else {
                    lam_off += a.lam[i];
                }
            }
        }
    }
    num = __builtin_fmaf(lam_off * a0, d, num);
    den = __builtin_fmaf(lam_off, a02, den);
    const float vv = num * __builtin_amdgcn_rcpf(den);  // hardware reciprocal, ~1 ulp
    // v n is the step per unit length; in voxels along each axis it is v n / h = v n 2 gs
    du[0] = vv * nxv * (2.f * a.gs[0]);
    du[1] = vv * nyv * (2.f * sy);
    du[2] = vv * nzv * (2.f * a.gs[2]);
}

// pair owning logical block L of a batched launch: prefix[q] <= L < prefix[q + 1]
__device__ __forceinline__ int pair_of(const int *prefix, int n, int L)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= L) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// one launch over the tiles of several pairs (each pair at its own level and size); the
// pair descriptors travel in the kernel-argument segment and are read with scalar loads

// Moving-mask occupancy of 8x8x8 bricks: OR of the mask bits over the brick grown by one
// voxel on its high side, so that a trilinear stencil whose base corner lies in the brick
// touches a structure only if the brick's entry is nonzero.
__global__ void __launch_bounds__(256) k_brick_occupancy(const uint8_t *__restrict__ bits, Dims d, Dims db,
                                                         uint8_t *__restrict__ occ)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= db.n()) return;
    const int bx = (int)(b % db.nx), by = (int)((b / db.nx) % db.ny), bz = (int)(b / ((int64_t)db.nx * db.ny));
    uint32_t o = 0;
    for (int l = 8 * bz; l <= min(8 * bz + 8, d.nz - 1); ++l)
        for (int j = 8 * by; j <= min(8 * by + 8, d.ny - 1); ++j)
            for (int i = 8 * bx; i <= min(8 * bx + 8, d.nx - 1); ++i)
                o |= bits[i + (int64_t)d.nx * (j + (int64_t)d.ny * l)];
    occ[b] = (uint8_t)o;
}

// ============================================================================
// Separable Gaussian (kernel 1) of u_c into u, sampled, radius R = ceil(3 sigma),
// normalised, clamped indices, followed by the warp of the moving image with the new u
// (kernel 4 on images).  A block owns a 64 x TY column tile and marches through the planes
// z0 - R .. z1 - 1 + R that its z pass needs (clamped: a plane past a volume end is the end
// plane again).  Each plane goes through three stages, one block-wide step apart: (a) its
// values (tile + R halo, prefetched into registers one step earlier) are stored into LDS, (b)
// filtered along x into a second LDS buffer, (c) filtered along y and pushed into a register
// ring of 2R + 1 planes that the z pass reads.  One step runs stage (a) of plane l, (b) of
// plane l - 1 and (c) of plane l - 2 on double-buffered LDS, so a step needs one barrier and
// its three stages' latencies overlap.  The warp of an output plane is issued after the plane's
// store and finished one step later, so its gathers overlap the next step's filtering.
// ============================================================================
template <int R, int TY, bool kAniso>
__device__ __forceinline__ void smooth_tile(const SmoothArgs &a, int L)
{
    constexpr int WD = kTileX + 2 * R, HT = TY + 2 * R, NT = kTileX * TY;
    constexpr int CELLS = HT * WD, NP = (CELLS + NT - 1) / NT;
    __shared__ float raw[2][3][HT][WD];
    __shared__ float xs[2][3][HT][kTileX];

    const int tid = threadIdx.x;
    const int tx = tid % kTileX, ty = tid / kTileX;
    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, nxy = nx * ny;
    const TileCoord tc = tile_of(TY, a.tz, a.d, L);
    const int x0 = tc.x0, y0 = tc.y0, z0 = tc.z0, z1 = tc.z1;
    // the Gaussians along x, y and z (y takes x's unless the voxel sizes differ)
    float wx[R + 1], wyv[R + 1], wz[R + 1];
#pragma unroll
    for (int m = 0; m <= R; ++m) {
        wx[m] = a.wx[m];
        if constexpr (kAniso) wyv[m] = a.wy[m];
        wz[m] = a.wz[m];
    }
    const float *wy = kAniso ? wyv : wx;

    const float *__restrict__ in0 = a.in[0];
    const float *__restrict__ in1 = a.in[1];
    const float *__restrict__ in2 = a.in[2];

    // staged cells of this thread (tile + R halo), as clamped in-plane offsets
    int coff[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int c = tid + j * NT;
        const int r = c / WD, q = c - r * WD;
        coff[j] = clampi(x0 - R + q, 0, nx - 1) + nx * clampi(y0 - R + r, 0, ny - 1);
    }
    float pre[NP][3];
    auto prefetch = [&](int p) {
        const int base = nxy * clampi(p, 0, nz - 1);
#pragma unroll
        for (int j = 0; j < NP; ++j)
            if (tid + j * NT < CELLS) {
                pre[j][0] = ldg(in0, base + coff[j]);
                pre[j][1] = ldg(in1, base + coff[j]);
                pre[j][2] = ldg(in2, base + coff[j]);
            }
    };

    float ring[3][2 * R + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m <= 2 * R; ++m) ring[k][m] = 0.f;

    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < nx && gy < ny;
    WarpPending wp;
    int wv = -1;
    const int lo = z0 - R, count = (z1 - z0) + 2 * R;  // planes lo .. lo + count - 1
    // Two blocks share a compute unit.  The SIMDs issue from the older block's waves first, so
    // left alone it finishes well before the younger one (measured on full launches: the
    // first-dispatched blocks end about 60 us of 400 earlier) and the unit then runs half its
    // waves.  The blocks of even and odd passes of the dispatcher over the 256 units take the
    // higher issue priority on alternate steps instead, so that both advance at one pace.
    const int pass = (blockIdx.x / kComputeUnits) & 1;
    prefetch(lo);
    for (int i = 0; i < count + 2; ++i) {
        if ((i + pass) & 1) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        // (a) plane lo + i into raw[i & 1], and the next plane's prefetch
        if (i < count) {
            const int sb = i & 1;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const int c = tid + j * NT;
                if (c < CELLS) {
                    const int r = c / WD, q = c - r * WD;
                    raw[sb][0][r][q] = pre[j][0];
                    raw[sb][1][r][q] = pre[j][1];
                    raw[sb][2][r][q] = pre[j][2];
                }
            }
            if (i + 1 < count) prefetch(lo + i + 1);
        }
        // (b) x pass of plane lo + i - 1
        if (i >= 1 && i <= count) {
            const int sb = (i - 1) & 1;
            for (int c = tid; c < HT * kTileX; c += NT) {
                const int r = c / kTileX, q = c - r * kTileX;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float t = wx[0] * raw[sb][k][r][q + R];
#pragma unroll
                    for (int m = 1; m <= R; ++m)
                        t = __builtin_fmaf(wx[m], raw[sb][k][r][q + R - m] + raw[sb][k][r][q + R + m], t);
                    xs[sb][k][r][q] = t;
                }
            }
        }
        // (c) y pass of plane lo + i - 2 into the ring; once the ring holds planes
        // z - R .. z + R, the z pass and the output of plane z = lo + i - 2 - R
        if (i >= 2) {
            const int sb = i & 1;  // ((i - 2) & 1)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float t = wy[0] * xs[sb][k][ty + R][tx];
#pragma unroll
                for (int m = 1; m <= R; ++m) t = __builtin_fmaf(wy[m], xs[sb][k][ty + R - m][tx] + xs[sb][k][ty + R + m][tx], t);
#pragma unroll
                for (int m = 0; m < 2 * R; ++m) ring[k][m] = ring[k][m + 1];
                ring[k][2 * R] = t;
            }
            if (wv >= 0) warp_finish(a.warp, wp, wv);
            wv = -1;
            if (i - 2 >= 2 * R && own) {
                const int z = lo + i - 2 - R;
                const int v = gx + nx * gy + nxy * z;
                float s3[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float t = wz[0] * ring[k][R];
#pragma unroll
                    for (int m = 1; m <= R; ++m) t = __builtin_fmaf(wz[m], ring[k][R - m] + ring[k][R + m], t);
                    s3[k] = t;
                    stg(a.out[k], v, t);
                }
                warp_issue(a.warp, gx, gy, z, s3[0], s3[1], s3[2], wp);
                wv = v;
            }
        }
        __syncthreads();
    }
    if (wv >= 0) warp_finish(a.warp, wp, wv);
}

template <int R, int TY, bool kAniso>
__global__ void __launch_bounds__(kTileX *TY) k_smooth_batch(SmoothBatch b)
{
    const int L = xcd_logical(blockIdx.x, b.prefix[b.n]);
    const int q = pair_of(b.prefix, b.n, L);
    if (b.d[q].stop) {  // the pair stopped after an earlier iteration: nothing to do
        const int s = *b.d[q].stop;
        if (s != 0 && s <= b.d[q].iter) return;
    }
    smooth_tile<R, TY, kAniso>(b.d[q], L - b.prefix[q]);
}

// ============================================================================
// One iteration up to the composite update, fused: kernels 2 and 3 (gradient and Eq.7) give
// du, kernel 1 smooths it with the fluid Gaussian (clamped indices), and kernel 4 composes
// the smoothed step s with the field: u_c(x) = s(x) + u(x + s(x)), u gathered trilinearly.
//
// A block owns a 64 x TY column tile and a chunk of z planes.  It marches through the
// planes z0 - R .. z1 - 1 + R that its z pass needs; for each distinct clamped plane it
// evaluates du on the tile + R halo (the cells the x and y passes read), straight into LDS,
// so du never goes to memory.  A halo cell is evaluated at its clamped voxel, which gives
// the clamped-index smoothing exactly.  The I0~ planes (and structure bits) of the stencils,
// tile + R + 1 halo, go through an LDS ring indexed by plane (three slots for 16-row tiles,
// four for smaller ones), loaded two planes ahead; the field's planes around the output plane
// (tile + 1 halo) go through a 3-slot ring for the compose gathers, with a global fallback
// when |s| >= 1.
// ============================================================================
// kMasked false: no pair of the launch has contour terms at its level (no structure bits, K~
// or contour weights in LDS, so the block needs less of it and of registers).
template <int R, int TY, bool kMasked, bool kAniso>
__device__ __forceinline__ void step_tile(const StepArgs &a, int L)
{
    constexpr int WD = kTileX + 2 * R, HT = TY + 2 * R, NT = kTileX * TY;
    constexpr int CELLS = HT * WD, NP = (CELLS + NT - 1) / NT;
    constexpr int WW = WD + 2, WH = HT + 2, WCELLS = WW * WH, NW = (WCELLS + NT - 1) / NT;
    constexpr int UW = kTileX + 2, UH = TY + 2, UCELLS = UW * UH, NU = (UCELLS + NT - 1) / NT;
    // LDS of the block (160 KiB at most): the structure bits as 32-bit words, which the force
    // reads faster than bytes (bytes for the widest radii), and, where the words leave room,
    // for the 16-row tiles (one block per CU: the slowest block sets the launch's time) K~
    // of three staged planes (the warped masked moving image of the one structure near a
    // cell), so that the force near a structure reads no memory.  (Smaller tiles keep their
    // LDS small so that more blocks share a CU.)  The I0~ and bit rings of the 16-row tiles
    // hold three planes (four for smaller tiles): a plane's slot is refilled once every wave
    // has passed the force of the plane above it.
    //
    // The u ring's row stride is padded to a multiple of the 32 LDS banks where that costs
    // neither the 32-bit bit words nor a block per CU: the compose's corner reads take rows
    // and planes that differ from lane to lane, and with the padded stride those rows and
    // planes fall into the same banks for the same column instead of colliding with the
    // neighbouring lanes' columns.  The padding columns then hold the squared metric terms
    // and the weight table.
    constexpr int kLdsMax = 160 * 1024, kSlots = TY == 16 ? 3 : 4;
    constexpr int UWP = (UW + 31) / 32 * 32, PADW = UWP - UW;
    static_assert(PADW > 0, "the u ring rows are padded to a multiple of 32");
    constexpr int kDqF = TY * kTileX, kLamF = 2 * kMaxStructs;  // floats of the metric terms, weights
    // (whole rows of padding for the metric terms, the last row's for the weights; only for
    // the 16-row tiles, where the 160 KiB are short)
    constexpr bool kSideFits = TY == 16 && PADW >= kLamF && (kDqF + PADW - 1) / PADW <= 9 * UH - 1;
    constexpr int kFixedB = 4 * (kSlots * WCELLS + 3 * HT * WD + 3 * HT * kTileX);  // I0~, du, x pass
    constexpr int kLdsU = kFixedB + 36 * UH * UW + 4 * (kDqF + kLamF);
    constexpr int kLdsP = kFixedB + 36 * UH * UWP + (kSideFits ? 0 : 4 * (kDqF + kLamF));
    constexpr int kFrWordsB = 4 * kSlots * WCELLS, kFrBytesB = kSlots * WCELLS;
    constexpr bool kWordsU = TY == 16 && kLdsU + kFrWordsB <= kLdsMax;
    constexpr bool kWordsP = TY == 16 && kLdsP + kFrWordsB <= kLdsMax;
    constexpr int kBlocksU = cmin(2048 / NT, kLdsMax / (kLdsU + (kMasked ? (kWordsU ? kFrWordsB : kFrBytesB) : 0)));
    constexpr int kBlocksP = cmin(2048 / NT, kLdsMax / (kLdsP + (kMasked ? (kWordsP ? kFrWordsB : kFrBytesB) : 0)));
    constexpr bool kPad = kWordsP == kWordsU && kBlocksP >= kBlocksU;
    constexpr bool kSideInPad = kPad && kSideFits;
    constexpr int US = kPad ? UWP : UW;  // u ring row stride
    constexpr int UPLANE = US * UH;      // and plane stride
    constexpr int kLdsBase = kPad ? kLdsP : kLdsU;
    constexpr bool kFr32 = TY == 16 && kLdsBase + kFrWordsB <= kLdsMax;
    constexpr bool kStageK = kMasked && TY == 16 && kLdsBase + kFrWordsB + 12 * WCELLS <= kLdsMax;
    using FrT = typename std::conditional<kFr32, uint32_t, uint8_t>::type;
    // One LDS buffer laid out by hand, in order of access density: the arrays read at many
    // constant offsets from one address come first, below 64 KiB, where those offsets fit the
    // LDS instructions' own offset field instead of costing an address add each.
    constexpr int kRawB = 4 * 3 * HT * WD, kXsB = 4 * 3 * HT * kTileX, kUsB = 4 * 9 * UPLANE;
    constexpr int kWrB = 4 * kSlots * WCELLS, kFrB = kMasked ? kSlots * WCELLS * (int)sizeof(FrT) : 4;
    constexpr int kKrB = kStageK ? 4 * 3 * WCELLS : 4, kSideB = kSideInPad ? 4 : 4 * (kDqF + kLamF);
    constexpr int oXs = kRawB, oUs = oXs + kXsB, oWr = oUs + kUsB, oFr = oWr + kWrB;
    constexpr int oKr = oFr + ((kFrB + 3) & ~3), oSide = oKr + kKrB, kLdsTotal = oSide + kSideB;
    static_assert(kLdsTotal <= kLdsMax, "LDS budget of the step kernel");
    __shared__ __attribute__((aligned(16))) char smem[kLdsTotal];
    auto raw = reinterpret_cast<float(*)[HT][WD]>(smem);            // du on the tile + R halo
    auto xs = reinterpret_cast<float(*)[HT][kTileX]>(smem + oXs);
    auto Us = reinterpret_cast<float(*)[3][UPLANE]>(smem + oUs);    // u planes z-1..z+1,
                                                                    // slot (p - z0 + 1) % 3
    auto Wr = reinterpret_cast<float(*)[WCELLS]>(smem + oWr);       // I0~ planes, slot = plane % 3
    auto Fr = reinterpret_cast<FrT(*)[WCELLS]>(smem + oFr);         // their stencil structure bits
    auto Kr = reinterpret_cast<float(*)[WCELLS]>(smem + oKr);       // K~ where the bits are
                                                                    // nonzero, slot = plane % 3
    // the squared metric terms of the tile's voxels, voxel d = row * 64 + column at dq[dq_at(d)],
    // and lambda_i with the sum of the other weights in index order (16 floats)
    float *const dq = reinterpret_cast<float *>(smem + (kSideInPad ? oUs : oSide));
    auto dq_at = [](int d) { return kSideInPad ? (d / PADW) * US + UW + d % PADW : d; };
    float *const lamt = kSideInPad ? reinterpret_cast<float *>(smem + oUs) + (9 * UH - 1) * US + UW
                                   : reinterpret_cast<float *>(smem + oSide) + kDqF;

    const int tid = threadIdx.x;
    const int tx = tid % kTileX, ty = tid / kTileX;
    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, nxy = nx * ny;
    const TileCoord tc = tile_of(TY, a.tz, a.d, L);
    const int x0 = tc.x0, y0 = tc.y0, z0 = tc.z0, z1 = tc.z1;
    const bool masked = kMasked && a.F != nullptr;
    const bool metric = a.partials != nullptr;
    // the Gaussians along x, y and z (y takes x's unless the voxel sizes differ)
    float wx[R + 1], wyv[R + 1], wz[R + 1];
#pragma unroll
    for (int m = 0; m <= R; ++m) {
        wx[m] = a.wx[m];
        if constexpr (kAniso) wyv[m] = a.wy[m];
        wz[m] = a.wz[m];
    }
    const float *wy = kAniso ? wyv : wx;

    // ---- I0~ / structure-bit ring (tile + R + 1 halo), clamped in-plane offsets
    int woff[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        const int c = tid + j * NT;
        const int r = c / WW, q = c - r * WW;
        woff[j] = clampi(x0 - R - 1 + q, 0, nx - 1) + nx * clampi(y0 - R - 1 + r, 0, ny - 1);
    }
    float pw[NW];
    uint32_t pf[NW];
    auto w_load = [&](int p) {  // p in [0, nz)
        const int base = nxy * p;
#pragma unroll
        for (int j = 0; j < NW; ++j)
            if (tid + j * NT < WCELLS) {
                pw[j] = ldg(a.wI0, base + woff[j]);
                pf[j] = masked ? ldg(a.F, base + woff[j]) : 0u;
            }
    };
    // w_put stores a loaded plane into its ring slot (once no wave reads the plane it replaces);
    // k_issue issues the K~ loads of the cells whose bits are nonzero, and k_store puts them
    // into the K~ ring once the plane they replace is no longer read and their latency is covered
    auto w_put = [&](int p) {
        const int sl = p % kSlots;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const int c = tid + j * NT;
            if (c < WCELLS) {
                Wr[sl][c] = pw[j];
                if constexpr (kMasked) Fr[sl][c] = (FrT)pf[j];
            }
        }
    };
    float pk[NW];
    uint32_t kpend = 0u;
    int kplane = 0;
    bool kwave = false;  // this wave has K~ loads pending
    auto k_issue = [&](int p) {
        if constexpr (kStageK) {
            kpend = 0u;
            kplane = p;
            uint32_t any = 0u;
#pragma unroll
            for (int j = 0; j < NW; ++j)
                if (tid + j * NT < WCELLS) any |= pf[j];
            kwave = masked && __ballot(any != 0u) != 0ull;  // (the same in every lane)
            if (kwave) {
                const int base = nxy * p;
#pragma unroll
                for (int j = 0; j < NW; ++j)
                    if (tid + j * NT < WCELLS && pf[j] != 0) {
                        pk[j] = ldg(a.K, base + woff[j]);
                        kpend |= 1u << j;
                    }
            }
        }
    };
    auto k_store = [&]() {
        if constexpr (kStageK) {
            if (kwave) {
                const int sl = kplane % 3;
#pragma unroll
                for (int j = 0; j < NW; ++j)
                    if ((kpend >> j) & 1u) Kr[sl][tid + j * NT] = pk[j];
                kpend = 0u;
                kwave = false;
            }
        }
    };

    // ---- du cells (tile + R halo): clamped voxel coordinates, target values one plane ahead
    int cgx[NP], cgy[NP], dqi[NP];
    uint32_t inside = 0;  // bit j: cell j is a voxel of the tile inside the volume
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int c = tid + j * NT;
        const int r = c / WD, q = c - r * WD;
        cgx[j] = clampi(x0 - R + q, 0, nx - 1);
        cgy[j] = clampi(y0 - R + r, 0, ny - 1);
        const bool tile = c < CELLS && r >= R && r < R + TY && q >= R && q < R + kTileX;
        dqi[j] = tile ? dq_at((r - R) * kTileX + (q - R)) : -1;
        if (tile && x0 + q - R < nx && y0 + r - R < ny) inside |= 1u << j;
    }
    float pt[NP];
    uint32_t ptb[NP], pur[NP];
    auto t_load = [&](int p) {
#pragma unroll
        for (int j = 0; j < NP; ++j)
            if (tid + j * NT < CELLS) {
                const int v = cgx[j] + nx * cgy[j] + nxy * p;
                pt[j] = ldg(a.T0, v);
                ptb[j] = masked ? ldg(a.tbits, v) : 0u;
                pur[j] = (metric && ((inside >> j) & 1u)) ? ldg(a.uroi, v) : 0u;
            }
    };

    // ---- u ring (tile + 1 halo) for the compose gathers
    int uoff[NU], uadr[NU];  // global offset and ring cell of each staged u cell
#pragma unroll
    for (int j = 0; j < NU; ++j) {
        const int c = tid + j * NT;
        const int r = c / UW, q = c - r * UW;
        uoff[j] = clampi(x0 - 1 + q, 0, nx - 1) + nx * clampi(y0 - 1 + r, 0, ny - 1);
        uadr[j] = r * US + q;
    }
    float upre[NU][3];
    auto u_load = [&](int p) {
        const int base = nxy * clampi(p, 0, nz - 1);
#pragma unroll
        for (int j = 0; j < NU; ++j)
            if (tid + j * NT < UCELLS) {
                upre[j][0] = ldg(a.u[0], base + uoff[j]);
                upre[j][1] = ldg(a.u[1], base + uoff[j]);
                upre[j][2] = ldg(a.u[2], base + uoff[j]);
            }
    };
    auto u_store = [&](int p) {
        const int sl = (p - z0 + 1) % 3;
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const int c = tid + j * NT;
            if (c < UCELLS) {
                Us[0][sl][uadr[j]] = upre[j][0];
                Us[1][sl][uadr[j]] = upre[j][1];
                Us[2][sl][uadr[j]] = upre[j][2];
            }
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

    // planes pa - 1 .. pa + 1 staged, pa + 2 in registers; plane q + 2 is staged once every
    // wave has evaluated plane q's du, into the slot of plane q - 1
    const int zs = z0 - R, ze = z1 - 1 + R;
    const int pa = max(zs, 0), pb = min(ze, nz - 1);
    w_load(max(pa - 1, 0));
    w_put(max(pa - 1, 0));
    k_issue(max(pa - 1, 0));
    k_store();
    w_load(pa);
    w_put(pa);
    k_issue(pa);
    k_store();
    w_load(min(pa + 1, nz - 1));
    w_put(min(pa + 1, nz - 1));
    k_issue(min(pa + 1, nz - 1));
    k_store();
    w_load(min(pa + 2, nz - 1));
    t_load(pa);
    u_load(z0 - 1);
    u_store(z0 - 1);
    u_load(z0);
    u_store(z0);
    u_load(z0 + 1);

    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < nx && gy < ny;
    const int ntx = (nx + kTileX - 1) / kTileX;
    const int cbase = (ty + 1) * US + tx + 1;  // this voxel's cell in a u ring plane
    float last[3] = {0.f, 0.f, 0.f};
    int prev = -1;
    if (kMasked && tid < kMaxStructs) {  // (the weights past k are zero; adding a zero is exact)
        float li = 0.f, off = 0.f;
#pragma unroll
        for (int m = 0; m < kMaxStructs; ++m) {
            const float lm = a.lam[m];
            li = m == tid ? lm : li;
            off += m == tid ? 0.f : lm;
        }
        lamt[tid] = li;
        lamt[kMaxStructs + tid] = off;
    }
    __syncthreads();
    for (int l = zs; l <= ze; ++l) {
        const int pc = clampi(l, 0, nz - 1);
        const int z = l - R;         // output plane once the ring is full
        const bool out = l >= z0 + R;
        float v3[3];
        if (pc != prev) {
            // ---- du on plane pc, tile + R halo
            const int s0 = pc % kSlots, sm = max(pc - 1, 0) % kSlots, sp = min(pc + 1, nz - 1) % kSlots;
            // K~ ring slots of this plane and the ones below and above (slot = plane % 3)
            const int kslots[3] = {(pc % 3) * WCELLS, (max(pc - 1, 0) % 3) * WCELLS,
                                   (min(pc + 1, nz - 1) % 3) * WCELLS};
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const int c = tid + j * NT;
                if (c < CELLS) {
                    const int cx = cgx[j], cy = cgy[j];
                    const int wo = (cy - (y0 - R - 1)) * WW + (cx - (x0 - R - 1));
                    float w7[7];
                    uint32_t f7[7];
                    w7[0] = Wr[s0][wo];
                    w7[1] = Wr[s0][wo - 1];
                    w7[2] = Wr[s0][wo + 1];
                    w7[3] = Wr[s0][wo - WW];
                    w7[4] = Wr[s0][wo + WW];
                    w7[5] = Wr[sm][wo];
                    w7[6] = Wr[sp][wo];
                    if (masked) {
                        f7[0] = Fr[s0][wo];
                        f7[1] = Fr[s0][wo - 1];
                        f7[2] = Fr[s0][wo + 1];
                        f7[3] = Fr[s0][wo - WW];
                        f7[4] = Fr[s0][wo + WW];
                        f7[5] = Fr[sm][wo];
                        f7[6] = Fr[sp][wo];
                    } else {
#pragma unroll
                        for (int q = 0; q < 7; ++q) f7[q] = 0u;
                    }
                    float du[3], d;
                    force_at<kStageK, WW, kAniso>(a, w7, f7, pt[j], ptb[j], cx, cy, pc, lamt,
                                          kStageK ? &Kr[0][0] + wo : nullptr, kslots, du, &d);
                    (&raw[0][0][0])[c] = du[0];  // cell c is row c / WD, column c % WD
                    (&raw[1][0][0])[c] = du[1];
                    (&raw[2][0][0])[c] = du[2];
                    if (metric && dqi[j] >= 0) {
                        const float e = d * a.inv_norm;
                        dq[dqi[j]] = pur[j] ? e * e : 0.f;
                    }
                }
            }
            // plane pc + 2 into the slot of plane pc - 1 once every wave is past this plane's
            // force (its K~ loads issued before the barrier); the loads are clamped into the
            // volume and issued unconditionally (a few unused planes at the chunk end) so that
            // no register copies are needed
            const bool stage = pc + 1 <= pb && pc + 2 <= nz - 1;
            if (stage) k_issue(pc + 2);
            __syncthreads();
            if (stage) w_put(pc + 2);
            w_load(min(pc + 3, nz - 1));
            t_load(min(pc + 1, nz - 1));
            for (int c = tid; c < HT * kTileX; c += NT) {
                const int r = c / kTileX, q = c - r * kTileX;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float s = wx[0] * raw[k][r][q + R];
#pragma unroll
                    for (int m = 1; m <= R; ++m)
                        s = __builtin_fmaf(wx[m], raw[k][r][q + R - m] + raw[k][r][q + R + m], s);
                    xs[k][r][q] = s;
                }
            }
            // stopping metric: one partial per 64-voxel row segment (a wave is one tile
            // row), a grouping that does not depend on the launch geometry
            if (metric && pc >= z0 && pc < z1 && gy < ny) {
                const float rs = wave_sum(dq[dq_at(ty * kTileX + tx)]);
                if (tx == 0) stg(a.partials, (pc * ny + gy) * ntx + x0 / kTileX, rs);
            }
            if (out) {
                u_store(z + 1);
                u_load(z + 2);
            }
            k_store();
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float s = wy[0] * xs[k][ty + R][tx];
#pragma unroll
                for (int m = 1; m <= R; ++m) s = __builtin_fmaf(wy[m], xs[k][ty + R - m][tx] + xs[k][ty + R + m][tx], s);
                v3[k] = s;
                last[k] = s;
            }
            prev = pc;
        } else {  // a clamped plane again (past a volume end): same xy-smoothed values
#pragma unroll
            for (int k = 0; k < 3; ++k) v3[k] = last[k];
            if (out) {
                __syncthreads();
                u_store(z + 1);
                u_load(z + 2);
                __syncthreads();
            }
        }
        push(v3);
        if (out && own) {
            const int v = gx + nx * gy + nxy * z;
            float s[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float t = wz[0] * ring[k][R];
#pragma unroll
                for (int m = 1; m <= R; ++m) t = __builtin_fmaf(wz[m], ring[k][R - m] + ring[k][R + m], t);
                s[k] = t;
            }
            // lower corner of the sample x + s relative to the voxel: with each offset in
            // {-1, 0} every corner lies in the ring.  The ring holds a one-cell halo staged at
            // clamped coordinates, so where the sample leaves the volume the two corners along
            // that axis hold the same value, their interpolation returns it exactly, and the
            // result equals the clamped sample (split_axis) without any clamping here.
            const float fx = floorf(s[0]), fy = floorf(s[1]), fz = floorf(s[2]);
            const bool near = __builtin_fabsf(fx + 0.5f) <= 0.5f && __builtin_fabsf(fy + 0.5f) <= 0.5f &&
                              __builtin_fabsf(fz + 0.5f) <= 0.5f;  // (NaN: not near)
            if (near) {
                // ring cells: the plane's slot base (uniform), then the row and column offset
                const int zs_m = ((z - z0) % 3) * UPLANE, zs_0 = ((z - z0 + 1) % 3) * UPLANE;
                const int zs_p = ((z - z0 + 2) % 3) * UPLANE;
                const int cell = cbase + (int)__builtin_fmaf(fy, (float)US, fx);
                const int i0 = (fz < 0.f ? zs_m : zs_0) + cell, i1 = (fz < 0.f ? zs_0 : zs_p) + cell;
                const float tx_ = s[0] - fx, ty_ = s[1] - fy, tz_ = s[2] - fz;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float *U = &Us[k][0][0];
                    float f[8];
                    f[0] = U[i0];
                    f[1] = U[i0 + 1];
                    f[2] = U[i0 + US];
                    f[3] = U[i0 + US + 1];
                    f[4] = U[i1];
                    f[5] = U[i1 + 1];
                    f[6] = U[i1 + US];
                    f[7] = U[i1 + US + 1];
                    stg(a.uc[k], v, s[k] + lerp8(f, tx_, ty_, tz_));
                }
            } else {
                const Corners q = corners(split_axis(gx, s[0], nx), split_axis(gy, s[1], ny),
                                          split_axis(z, s[2], nz), nx, nxy);
#pragma unroll
                for (int k = 0; k < 3; ++k) stg(a.uc[k], v, s[k] + trilinear(a.u[k], q));
            }
        }
    }
}

template <int R, int TY, bool kMasked, bool kAniso>
__global__ void __launch_bounds__(kTileX *TY) k_step_batch(StepBatch b)
{
    const int L = xcd_logical(blockIdx.x, b.prefix[b.n]);
    const int q = pair_of(b.prefix, b.n, L);
    if (b.d[q].stop) {  // the pair stopped after an earlier iteration: nothing to do
        const int s = *b.d[q].stop;
        if (s != 0 && s <= b.d[q].iter) return;
    }
    step_tile<R, TY, kMasked, kAniso>(b.d[q], L - b.prefix[q]);
}

// Warp of the moving image with the field at the start of a level (the smoothing of u
// produces it for every later iteration).
__global__ void __launch_bounds__(256) k_warp_init(WarpArgs w, Field3 u)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= w.d.n()) return;
    const int i = (int)(idx % w.d.nx);
    const int j = (int)((idx / w.d.nx) % w.d.ny);
    const int l = (int)(idx / ((int64_t)w.d.nx * w.d.ny));
    WarpPending p;
    warp_issue(w, i, j, l, u.p[0][idx], u.p[1][idx], u.p[2][idx], p);
    warp_finish(w, p, (int)idx);
}

// ============================================================================
// Stopping metric: delta = sqrt(sum of the per-block partials / |UROI|), summed in a fixed
// order in double precision (kernel 5).
// ============================================================================
__global__ void __launch_bounds__(256) k_delta_finalize_batch(DeltaBatch b)
{
    const DeltaJob &j = b.d[blockIdx.x];
    if (j.stop && *j.stop) return;  // stopped at an earlier iteration
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < j.nparts; i += 256) s += (double)j.partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t c = *j.count;
        const double delta = c > 0 ? sqrt(red[0] / (double)c) : 0.0;
        j.hist[j.n] = delta;
        // stopping rule on the device: delta_{n-W} - delta_n <= eps after every W iterations
        if (j.window > 0 && (j.n + 1) % j.window == 0 && j.n - j.window >= 0 &&
            j.hist[j.n - j.window] - delta <= j.eps)
            *j.stop = j.n + 1;
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

// Structure bits at pyramid level l (contour terms below the finest level): the bits of the
// finest voxel that coarse voxel (i, j, k) stands for, (2^l i, 2^l j, 2^l k), the voxel every
// restriction step keeps.  One thread per coarse voxel; dc = level_dims(d0, l).
__global__ void __launch_bounds__(256) k_level_bits(const uint8_t *__restrict__ bits0, Dims d0, int shift,
                                                    uint8_t *__restrict__ out, Dims dc)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= dc.n()) return;
    const int i = (int)(v % dc.nx);
    const int j = (int)((v / dc.nx) % dc.ny);
    const int l = (int)(v / ((int64_t)dc.nx * dc.ny));
    const int64_t f = (int64_t)(i << shift) + (int64_t)d0.nx * ((int64_t)(j << shift) + (int64_t)d0.ny * (l << shift));
    out[v] = bits0[f];
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

int tile_blocks(Dims d, int ty, int tz) { return tiles_xy(d, ty) * ((d.nz + tz - 1) / tz); }

// one launch per (radius, tile rows, contour terms in the launch, x and y voxel sizes
// differ) instantiation
template <int TY, bool kMasked, bool kAniso>
static hipError_t step_batch_ty(const StepBatch &b, int radius, hipStream_t s)
{
    const dim3 grid(b.prefix[b.n]), block(kTileX * TY);
    switch (radius) {
    case 0: hipLaunchKernelGGL((k_step_batch<0, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    case 1: hipLaunchKernelGGL((k_step_batch<1, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    case 2: hipLaunchKernelGGL((k_step_batch<2, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    case 3: hipLaunchKernelGGL((k_step_batch<3, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    case 4: hipLaunchKernelGGL((k_step_batch<4, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    case 5: hipLaunchKernelGGL((k_step_batch<5, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    case 6: hipLaunchKernelGGL((k_step_batch<6, TY, kMasked, kAniso>), grid, block, 0, s, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int TY>
static hipError_t step_batch_flags(const StepBatch &b, int radius, bool masked, bool aniso, hipStream_t s)
{
    if (aniso) return masked ? step_batch_ty<TY, true, true>(b, radius, s) : step_batch_ty<TY, false, true>(b, radius, s);
    return masked ? step_batch_ty<TY, true, false>(b, radius, s) : step_batch_ty<TY, false, false>(b, radius, s);
}

// the y axis has its own scale and taps (the general instantiation) only where they differ
// from x's: square in-plane voxels run the instantiation that reuses x's
static bool differs(const float *a, const float *b, int n)
{
    for (int i = 0; i < n; ++i)
        if (a[i] != b[i]) return true;
    return false;
}

hipError_t launch_step_batch(const StepBatch &b, int radius, int ty, hipStream_t s)
{
    if (b.n < 1 || b.n > kBatchStep || b.prefix[b.n] < 1) return hipErrorInvalidValue;
    bool masked = false, aniso = false;  // any pair of the launch with contour terms at its
                                         // level; with x and y voxel sizes that differ
    for (int i = 0; i < b.n; ++i) {
        masked = masked || b.d[i].F != nullptr;
        aniso = aniso || b.d[i].gs[0] != b.d[i].gs[1] || b.d[i].far_c[0] != b.d[i].far_c[1] ||
                b.d[i].gs2[0] != b.d[i].gs2[1] || differs(b.d[i].wx, b.d[i].wy, kMaxRadius + 1);
    }
    switch (ty) {
    case 4: return step_batch_flags<4>(b, radius, masked, aniso, s);
    case 8: return step_batch_flags<8>(b, radius, masked, aniso, s);
    case 16: return step_batch_flags<16>(b, radius, masked, aniso, s);
    default: return hipErrorInvalidValue;
    }
}

template <int TY, bool kAniso>
static hipError_t smooth_batch_ty(const SmoothBatch &b, int radius, hipStream_t s)
{
    const dim3 grid(b.prefix[b.n]), block(kTileX * TY);
    switch (radius) {
    case 0: hipLaunchKernelGGL((k_smooth_batch<0, TY, kAniso>), grid, block, 0, s, b); break;
    case 1: hipLaunchKernelGGL((k_smooth_batch<1, TY, kAniso>), grid, block, 0, s, b); break;
    case 2: hipLaunchKernelGGL((k_smooth_batch<2, TY, kAniso>), grid, block, 0, s, b); break;
    case 3: hipLaunchKernelGGL((k_smooth_batch<3, TY, kAniso>), grid, block, 0, s, b); break;
    case 4: hipLaunchKernelGGL((k_smooth_batch<4, TY, kAniso>), grid, block, 0, s, b); break;
    case 5: hipLaunchKernelGGL((k_smooth_batch<5, TY, kAniso>), grid, block, 0, s, b); break;
    case 6: hipLaunchKernelGGL((k_smooth_batch<6, TY, kAniso>), grid, block, 0, s, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_smooth_batch(const SmoothBatch &b, int radius, int ty, hipStream_t s)
{
    if (b.n < 1 || b.n > kBatchSmooth || b.prefix[b.n] < 1) return hipErrorInvalidValue;
    bool aniso = false;
    for (int i = 0; i < b.n; ++i) aniso = aniso || differs(b.d[i].wx, b.d[i].wy, kMaxRadius + 1);
    switch (ty) {
    case 4: return aniso ? smooth_batch_ty<4, true>(b, radius, s) : smooth_batch_ty<4, false>(b, radius, s);
    case 8: return aniso ? smooth_batch_ty<8, true>(b, radius, s) : smooth_batch_ty<8, false>(b, radius, s);
    case 16: return aniso ? smooth_batch_ty<16, true>(b, radius, s) : smooth_batch_ty<16, false>(b, radius, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_warp_init(const WarpArgs &w, const float *const u[3], hipStream_t s)
{
    Field3 f{{u[0], u[1], u[2]}};
    hipLaunchKernelGGL(k_warp_init, dim3(blocks_for(w.d.n(), 256)), dim3(256), 0, s, w, f);
    return hipGetLastError();
}

hipError_t launch_delta_batch(const DeltaBatch &b, hipStream_t s)
{
    if (b.n < 1 || b.n > kBatchDelta) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_delta_finalize_batch, dim3(b.n), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_brick_occupancy(const uint8_t *bits, Dims d, uint8_t *occ, hipStream_t s)
{
    const Dims db = brick_dims(d);
    hipLaunchKernelGGL(k_brick_occupancy, dim3(blocks_for(db.n(), 256)), dim3(256), 0, s, bits, d, db, occ);
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

hipError_t launch_level_bits(const uint8_t *bits0, Dims d0, int level, uint8_t *out, Dims dc, hipStream_t s)
{
    if (level < 1 || level >= 31) return hipErrorInvalidValue;
    // every kept index 2^l (ceil(n / 2^l) - 1) is below n
    if ((((int64_t)dc.nx - 1) << level) >= d0.nx || (((int64_t)dc.ny - 1) << level) >= d0.ny ||
        (((int64_t)dc.nz - 1) << level) >= d0.nz)
        return hipErrorInvalidValue;
    if (dc.n() == 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_bits, dim3(blocks_for(dc.n(), 256)), dim3(256), 0, s, bits0, d0, level, out, dc);
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
