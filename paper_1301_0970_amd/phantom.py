"""Seeded synthetic CT registration pairs.

The paper evaluates on clinical planning/treatment CT pairs of the head and neck and
the pelvis (section 2.3); that data is not available, so these generators stand in
for it with the same shapes, intensity ranges (air -1000 HU, soft tissue ~40 HU,
bone ~1200-1500 HU), low-contrast delineated structures and deformation magnitudes.

This module holds none of the registration arithmetic.  It draws a piecewise-constant
phantom ``P`` (ellipsoids), a smooth forward deformation ``d`` (a sum of Gaussian
bumps, optionally a radial bulge), and returns

    target T0(x) = P(x)        + noise_T        target masks n_i(x) = [x in E_i]
    moving I0(y) = P(y + d(y)) + noise_I        moving masks m_i(y) = [y + d(y) in E_i]

so that the registration field ``u`` with ``I0(x + u(x)) ~ T0(x)`` is the fixed point
``u* = -d(x + u*)`` (:func:`ground_truth_u`).  Both the HIP path and the oracle are
fed from here; neither imports the other.

Arrays are x-fastest: a volume has numpy shape ``(nz, ny, nx)``; a displacement field
has shape ``(3, nz, ny, nx)`` with components ordered (x, y, z), in voxel units.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 13010970

AIR_HU = -1000.0
BODY_HU = 40.0


def seed_for(config: int, pair: int = 0) -> int:
    """Seed of pair ``pair`` of workload number ``config`` (1..5)."""
    return SEED_BASE + 1000 * config + pair


@dataclasses.dataclass
class Ellipsoid:
    center: Tuple[float, float, float]  # (x, y, z) voxels
    semi: Tuple[float, float, float]    # semi-axes (x, y, z) voxels
    value: float                        # HU painted inside

    def bbox(self, dims, margin: float = 0.0):
        """Index ranges (z, y, x) slices covering the ellipsoid plus ``margin``."""
        sl = []
        for a in (2, 1, 0):
            lo = int(math.floor(self.center[a] - self.semi[a] - margin))
            hi = int(math.ceil(self.center[a] + self.semi[a] + margin)) + 1
            sl.append(slice(max(lo, 0), min(hi, dims[a])))
        return tuple(sl)

    def inside(self, px, py, pz):
        q = ((px - self.center[0]) / self.semi[0]) ** 2
        q = q + ((py - self.center[1]) / self.semi[1]) ** 2
        q = q + ((pz - self.center[2]) / self.semi[2]) ** 2
        return q <= 1.0


@dataclasses.dataclass
class Deformation:
    """Forward deformation d(y) = scale * sum_b a_b exp(-|y-c_b|^2 / 2 w_b^2) + bulge."""
    centers: np.ndarray   # (B, 3)
    widths: np.ndarray    # (B,)
    amps: np.ndarray      # (B, 3)
    scale: float
    bulge_center: Optional[Tuple[float, float, float]] = None
    bulge_rho: float = 0.0
    bulge_peak: float = 0.0

    def at(self, px, py, pz):
        """d evaluated at arbitrary points (broadcastable float64 arrays)."""
        px = np.asarray(px, np.float64)
        py = np.asarray(py, np.float64)
        pz = np.asarray(pz, np.float64)
        shape = np.broadcast(px, py, pz).shape
        dx = np.zeros(shape)
        dy = np.zeros(shape)
        dz = np.zeros(shape)
        for c, w, a in zip(self.centers, self.widths, self.amps):
            g = np.exp(-((px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2) / (2.0 * w * w))
            dx += a[0] * g
            dy += a[1] * g
            dz += a[2] * g
        dx *= self.scale
        dy *= self.scale
        dz *= self.scale
        if self.bulge_center is not None:
            rx = px - self.bulge_center[0]
            ry = py - self.bulge_center[1]
            rz = pz - self.bulge_center[2]
            r2 = rx * rx + ry * ry + rz * rz
            rho2 = self.bulge_rho ** 2
            # peak * (r/rho) * exp((1 - r^2/rho^2)/2) * r_hat  ==  peak/rho * exp(..) * r_vec
            f = self.bulge_peak / self.bulge_rho * np.exp(0.5 * (1.0 - r2 / rho2))
            dx += f * rx
            dy += f * ry
            dz += f * rz
        return dx, dy, dz

    def on_grid(self, dims, dtype=np.float32):
        """d on the full grid, using the separability of each bump; (3, nz, ny, nx)."""
        nx, ny, nz = dims
        x = np.arange(nx, dtype=np.float64)
        y = np.arange(ny, dtype=np.float64)
        z = np.arange(nz, dtype=np.float64)
        out = np.zeros((3, nz, ny, nx), dtype=dtype)
        for c, w, a in zip(self.centers, self.widths, self.amps):
            ex = np.exp(-((x - c[0]) ** 2) / (2 * w * w)).astype(dtype)
            ey = np.exp(-((y - c[1]) ** 2) / (2 * w * w)).astype(dtype)
            ez = np.exp(-((z - c[2]) ** 2) / (2 * w * w)).astype(dtype)
            g = ez[:, None, None] * (ey[:, None] * ex[None, :])[None, :, :]
            for comp in range(3):
                out[comp] += dtype(a[comp] * self.scale) * g
        if self.bulge_center is not None:
            rho = self.bulge_rho
            # the bulge is negligible beyond ~6 rho from its centre
            e = Ellipsoid(self.bulge_center, (6 * rho, 6 * rho, 6 * rho), 0.0)
            sl = e.bbox(dims)
            zz, yy, xx = np.meshgrid(z[sl[0]], y[sl[1]], x[sl[2]], indexing="ij")
            bx, by, bz = self._bulge_only(xx, yy, zz)
            out[0][sl] += bx.astype(dtype)
            out[1][sl] += by.astype(dtype)
            out[2][sl] += bz.astype(dtype)
        return out

    def _bulge_only(self, px, py, pz):
        rx = px - self.bulge_center[0]
        ry = py - self.bulge_center[1]
        rz = pz - self.bulge_center[2]
        r2 = rx * rx + ry * ry + rz * rz
        f = self.bulge_peak / self.bulge_rho * np.exp(0.5 * (1.0 - r2 / self.bulge_rho ** 2))
        return f * rx, f * ry, f * rz


@dataclasses.dataclass
class Pair:
    """One registration problem.  Volumes are float32 (nz, ny, nx); masks uint8 (k, nz, ny, nx)."""
    name: str
    target: np.ndarray
    moving: np.ndarray
    target_masks: np.ndarray
    moving_masks: np.ndarray
    signs: Tuple[int, ...]
    sigma: float
    levels: int
    iters: Tuple[int, ...]          # per level, index 0 = finest
    seed: int
    deformation: Deformation
    structures: List[Ellipsoid]
    phantom: List[Ellipsoid]

    @property
    def dims(self) -> Tuple[int, int, int]:
        nz, ny, nx = self.target.shape
        return (nx, ny, nz)

    @property
    def k(self) -> int:
        return int(self.target_masks.shape[0])

    @property
    def voxels(self) -> int:
        return int(self.target.size)

    def voxel_iterations(self) -> int:
        """sum over levels of N_level * iters_level, with level dims ceil(n/2) per level."""
        dims = self.dims
        total = 0
        for lv in range(self.levels):
            total += dims[0] * dims[1] * dims[2] * self.iters[lv]
            dims = tuple((n + 1) // 2 for n in dims)
        return total


# ----------------------------------------------------------------------------------
# drawing helpers


def _rng(seed: int, attempt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, attempt]))


def _draw_deformation(rng, dims, amp, n_bumps=8) -> Deformation:
    nx, ny, nz = dims
    n = np.array([nx, ny, nz], np.float64)
    centers = rng.uniform(0.2, 0.8, size=(n_bumps, 3)) * (n - 1)
    widths = rng.uniform(0.15, 0.3, size=n_bumps) * float(min(dims))
    dirs = rng.standard_normal((n_bumps, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    mags = rng.uniform(0.5, 1.0, size=n_bumps)
    amps = dirs * mags[:, None]
    dfm = Deformation(centers, widths, amps, 1.0)
    # rescale so that max |d| over a coarse grid equals amp
    gx, gy, gz = _coarse_grid(dims)
    dx, dy, dz = dfm.at(gx, gy, gz)
    mx = float(np.sqrt(dx * dx + dy * dy + dz * dz).max())
    dfm.scale = amp / mx if mx > 0 else 0.0
    return dfm


def _coarse_grid(dims, max_pts=40):
    axes = []
    for n in dims:
        step = max(1, int(math.ceil(n / max_pts)))
        axes.append(np.arange(0, n, step, dtype=np.float64))
    gz, gy, gx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return gx, gy, gz


def min_jacobian_det(dfm: Deformation, dims, h: float = 0.5) -> float:
    """min over a coarse grid of det(I + grad d), by central differences of the analytic d."""
    gx, gy, gz = _coarse_grid(dims)
    cols = []
    for e in ((h, 0, 0), (0, h, 0), (0, 0, h)):
        p = dfm.at(gx + e[0], gy + e[1], gz + e[2])
        m = dfm.at(gx - e[0], gy - e[1], gz - e[2])
        cols.append([(p[i] - m[i]) / (2 * h) for i in range(3)])
    # J[i][j] = d d_i / d x_j + delta_ij
    J = [[cols[j][i] + (1.0 if i == j else 0.0) for j in range(3)] for i in range(3)]
    det = (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
           - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
           + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))
    return float(det.min())


def _paint(dims, ellipsoids: Sequence[Ellipsoid], disp=None, dmax=0.0):
    """Evaluate the piecewise-constant phantom at x (disp None) or at x + disp(x)."""
    nx, ny, nz = dims
    vol = np.full((nz, ny, nx), AIR_HU, dtype=np.float32)
    for e in ellipsoids:
        sl = e.bbox(dims, margin=dmax + 1.0)
        ins = _inside_on(e, sl, disp)
        vol[sl][ins] = np.float32(e.value)
    return vol


def _inside_on(e: Ellipsoid, sl, disp):
    z = np.arange(sl[0].start, sl[0].stop, dtype=np.float64)[:, None, None]
    y = np.arange(sl[1].start, sl[1].stop, dtype=np.float64)[None, :, None]
    x = np.arange(sl[2].start, sl[2].stop, dtype=np.float64)[None, None, :]
    if disp is not None:
        x = x + disp[0][sl]
        y = y + disp[1][sl]
        z = z + disp[2][sl]
    return e.inside(x, y, z)


def _mask(dims, e: Ellipsoid, disp=None, dmax=0.0):
    nx, ny, nz = dims
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    sl = e.bbox(dims, margin=dmax + 1.0)
    m[sl] = _inside_on(e, sl, disp).astype(np.uint8)
    return m


def _disjoint(c, s, placed, pad=2.0):
    """True when the padded bounding boxes of (c, s) and every placed ellipsoid are disjoint."""
    for e in placed:
        if all(abs(c[a] - e.center[a]) < s[a] + e.semi[a] + pad for a in range(3)):
            return False
    return True


def _place_structures(rng, dims, body: Ellipsoid, count, semi_lo, semi_hi, contrast,
                      avoid: Sequence[Ellipsoid], fixed_semis=()):
    """Disjoint structure ellipsoids inside ``body``, away from ``avoid``."""
    placed: List[Ellipsoid] = []
    blockers = list(avoid)
    for i in range(count):
        for _ in range(2000):
            if i < len(fixed_semis):
                semi = tuple(float(v) for v in fixed_semis[i])
            else:
                semi = tuple(float(v) for v in rng.uniform(semi_lo, semi_hi, size=3))
            c = tuple(float(body.center[a] + rng.uniform(-0.6, 0.6) * max(body.semi[a] - semi[a], 0.0))
                      for a in range(3))
            inside = all(abs(c[a] - body.center[a]) + semi[a] <= body.semi[a] * 0.95 for a in range(3))
            if inside and _disjoint(c, semi, blockers):
                val = BODY_HU + float(contrast(rng))
                e = Ellipsoid(c, semi, val)
                placed.append(e)
                blockers.append(e)
                break
        else:  # pragma: no cover - geometry always leaves room at these sizes
            raise RuntimeError("could not place structure %d" % i)
    return placed


def _texture_at(waves, body: Ellipsoid, px, py, pz):
    """Smooth texture sum_j A_j cos(k_j . p + phi_j), only inside the body ellipsoid."""
    t = np.zeros(np.broadcast(px, py, pz).shape, np.float64)
    for a, kx, ky, kz, ph in waves:
        t += a * np.cos(kx * px + ky * py + kz * pz + ph)
    return np.where(body.inside(px, py, pz), t, 0.0)


def _draw_texture(rng, amp_hu, n_waves=6, wavelength=(6.0, 16.0)):
    waves = []
    for _ in range(n_waves):
        direction = rng.standard_normal(3)
        direction /= np.linalg.norm(direction)
        kv = direction * (2 * math.pi / rng.uniform(*wavelength))
        waves.append((amp_hu / math.sqrt(n_waves), kv[0], kv[1], kv[2], rng.uniform(0, 2 * math.pi)))
    return waves


def _assemble(name, seed, dims, phantom, structures, dfm, noise_sigma, sigma, levels, iters,
              rng, texture=None) -> Pair:
    disp = dfm.on_grid(dims, np.float32)
    mag = np.sqrt((disp.astype(np.float64) ** 2).sum(axis=0))
    dmax = float(mag.max())
    layers = list(phantom) + [e for e in structures if all(e is not p for p in phantom)]
    target = _paint(dims, layers)
    moving = _paint(dims, layers, disp, dmax)
    nx, ny, nz = dims
    if texture is not None:
        z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                              np.arange(nx, dtype=np.float64), indexing="ij")
        target += _texture_at(texture, phantom[0], x, y, z).astype(np.float32)
        moving += _texture_at(texture, phantom[0], x + disp[0], y + disp[1], z + disp[2]).astype(np.float32)
    target += (rng.standard_normal((nz, ny, nx), dtype=np.float32) * np.float32(noise_sigma))
    moving += (rng.standard_normal((nz, ny, nx), dtype=np.float32) * np.float32(noise_sigma))
    k = len(structures)
    tm = np.zeros((k, nz, ny, nx), np.uint8)
    mm = np.zeros((k, nz, ny, nx), np.uint8)
    for i, e in enumerate(structures):
        tm[i] = _mask(dims, e)
        mm[i] = _mask(dims, e, disp, dmax)
    return Pair(name, target, moving, tm, mm, tuple([1] * k), float(sigma), int(levels),
                tuple(int(v) for v in iters), seed, dfm, list(structures), list(phantom))


def _deformation_with_det_check(seed, dims, amp):
    for attempt in range(64):
        rng = _rng(seed, attempt)
        dfm = _draw_deformation(rng, dims, amp)
        if min_jacobian_det(dfm, dims) >= 0.2:
            return dfm, rng
    raise RuntimeError("no admissible deformation")  # pragma: no cover


# ----------------------------------------------------------------------------------
# the workloads


def plain_pair(dims=(64, 64, 32), seed=None, amp=4.0, noise=20.0, iters=100, sigma=1.0,
               levels=1, texture_hu=0.0) -> Pair:
    """Three nested ellipsoids (40 / 200 / 1500 HU) in air, one structure (the 200 HU one).
    ``texture_hu`` > 0 adds a smooth texture of that amplitude inside the body."""
    seed = seed_for(1) if seed is None else seed
    dfm, rng = _deformation_with_det_check(seed, dims, amp)
    n = np.array(dims, np.float64)
    ctr = tuple(float(v) for v in (n - 1) / 2)
    body = Ellipsoid(ctr, tuple(0.42 * n), BODY_HU)
    mid = Ellipsoid(ctr, tuple(0.25 * n), 200.0)
    inner = Ellipsoid(ctr, tuple(rng.uniform(0.08, 0.10, size=3) * n), 1500.0)
    tex = _draw_texture(rng, texture_hu) if texture_hu > 0 else None
    return _assemble("plain", seed, dims, [body, mid, inner], [mid], dfm, noise, sigma, levels,
                     (iters,) * levels, rng, texture=tex)


def head_neck_pair(dims=(256, 256, 128), seed=None, amp=8.0, noise=30.0, k=5,
                   levels=3, iters=100, sigma=1.5) -> Pair:
    """Head-and-neck-like: body, two bones, airway, ``k`` low-contrast (+10..30 HU) structures."""
    seed = seed_for(2) if seed is None else seed
    dfm, rng = _deformation_with_det_check(seed, dims, amp)
    n = np.array(dims, np.float64)
    c = (n - 1) / 2
    body = Ellipsoid(tuple(c), (0.42 * n[0], 0.44 * n[1], 0.46 * n[2]), BODY_HU)
    vert = Ellipsoid((c[0], c[1] + 0.22 * n[1], c[2]), (0.07 * n[0], 0.07 * n[1], 0.40 * n[2]), 1200.0)
    jaw = Ellipsoid((c[0], c[1] - 0.25 * n[1], c[2] + 0.18 * n[2]), (0.22 * n[0], 0.05 * n[1], 0.08 * n[2]), 1200.0)
    airway = Ellipsoid((c[0], c[1] + 0.05 * n[1], c[2]), (0.035 * n[0], 0.035 * n[1], 0.42 * n[2]), AIR_HU)
    s = min(dims) / 128.0
    structs = _place_structures(rng, dims, body, k, 8 * s, 20 * s, lambda r: r.uniform(10, 30),
                                [vert, jaw, airway])
    return _assemble("head_neck", seed, dims, [body, vert, jaw, airway], structs, dfm, noise,
                     sigma, levels, (iters,) * levels, rng)


def pelvis_pair(dims=(512, 512, 128), seed=None, amp=12.0, noise=40.0, k=8, levels=3,
                iters=150, sigma=1.0, bulge=5.0) -> Pair:
    """Pelvis-like: body, femoral heads, bladder-/rectum-like and smaller +15 HU structures,
    plus a radial bulge of peak ``bulge`` voxels centred on the bladder."""
    seed = seed_for(3) if seed is None else seed
    dfm, rng = _deformation_with_det_check(seed, dims, amp)
    n = np.array(dims, np.float64)
    c = (n - 1) / 2
    body = Ellipsoid(tuple(c), (0.45 * n[0], 0.34 * n[1], 0.48 * n[2]), BODY_HU)
    r_head = 0.05 * n[0]
    fem_l = Ellipsoid((c[0] - 0.30 * n[0], c[1], c[2] - 0.15 * n[2]), (r_head, r_head, min(r_head, 0.2 * n[2])), 1200.0)
    fem_r = Ellipsoid((c[0] + 0.30 * n[0], c[1], c[2] - 0.15 * n[2]), (r_head, r_head, min(r_head, 0.2 * n[2])), 1200.0)
    s = min(dims) / 128.0
    sxy = min(dims[0], dims[1]) / 512.0
    fixed = []
    if k >= 1:
        fixed.append((40 * sxy, 30 * sxy, 20 * s))   # bladder-like
    if k >= 2:
        fixed.append((12 * sxy, 12 * sxy, 40 * s))   # rectum-like
    structs = _place_structures(rng, dims, body, k, 6 * s, 14 * s, lambda r: 15.0,
                                [fem_l, fem_r], fixed_semis=fixed)
    if bulge > 0 and k >= 1:
        b = structs[0]
        dfm.bulge_center = b.center
        dfm.bulge_rho = float(np.prod(b.semi) ** (1.0 / 3.0))
        dfm.bulge_peak = float(bulge)
    return _assemble("pelvis", seed, dims, [body, fem_l, fem_r], structs, dfm, noise, sigma,
                     levels, (iters,) * levels, rng)


BATCH_XY = (128, 192, 256, 384, 512)


def batch_specs(n_pairs=32, config=4, seed_base=None):
    """Sizes and structure counts of the uneven batch: x, y from BATCH_XY, z in [64, 160],
    k in [1, 8], alternating head-and-neck-like and pelvis-like phantoms."""
    specs = []
    for p in range(n_pairs):
        seed = (seed_for(config, p) if seed_base is None else seed_base + p)
        rng = _rng(seed, 1000)
        nx = int(rng.choice(BATCH_XY))
        ny = int(rng.choice(BATCH_XY))
        nz = int(rng.integers(64, 161))
        k = int(rng.integers(1, 9))
        specs.append(dict(seed=seed, dims=(nx, ny, nz), k=k,
                          style="head_neck" if p % 2 == 0 else "pelvis"))
    return specs


def from_spec(spec, levels=3, iters=100, amp=8.0) -> Pair:
    if spec["style"] == "head_neck":
        return head_neck_pair(dims=spec["dims"], seed=spec["seed"], amp=amp, k=spec["k"],
                              levels=levels, iters=iters)
    return pelvis_pair(dims=spec["dims"], seed=spec["seed"], amp=amp, k=spec["k"],
                       levels=levels, iters=iters, bulge=0.0)


def batch_pairs(n_pairs=32, levels=3, iters=100) -> List[Pair]:
    return [from_spec(s, levels, iters) for s in batch_specs(n_pairs)]


def serve_schedule(rate=4.0, duration=120.0, seed=None):
    """Open-loop Poisson arrival times (seconds) and the pair spec of each request."""
    seed = seed_for(5) if seed is None else seed
    rng = _rng(seed, 0)
    t = 0.0
    times = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        times.append(t)
    specs = batch_specs(len(times), config=5)
    return times, specs


def make(config: str, **kw) -> Pair:
    """Named workloads: 'plain' (64x64x32), 'head_neck' (256x256x128), 'pelvis' (512x512x128)."""
    return {"plain": plain_pair, "head_neck": head_neck_pair, "pelvis": pelvis_pair}[config](**kw)


def ground_truth_u(pair: Pair, iters: int = 60) -> np.ndarray:
    """u* = -d(x + u*) by fixed-point iteration on the analytic deformation; (3, nz, ny, nx) f64."""
    nx, ny, nz = pair.dims
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    for _ in range(iters):
        dx, dy, dz = pair.deformation.at(x + u[0], y + u[1], z + u[2])
        u[0], u[1], u[2] = -dx, -dy, -dz
    return u


def random_smooth_field(dims, amp, seed, n_bumps=6) -> np.ndarray:
    """A seeded smooth displacement field (3, nz, ny, nx) float32 of max magnitude ~amp,
    used as a stand-in current iterate u^n for single-step comparisons."""
    dfm = _draw_deformation(_rng(seed, 7), dims, amp, n_bumps)
    return dfm.on_grid(dims, np.float32)
