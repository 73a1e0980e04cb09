"""Evaluation of a registration result, section 2.3 of the paper (plain numpy).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test suite and the benchmark's
CPU baseline may call it, the library never does.

What section 2.3 measures, with the readings taken where it is silent:
  * intensity: RMS-ID = sqrt(mean((I0~ - T0)^2)) and Pearson's CC between the deformed moving
    image I0~ = I0 o u and the target, over the whole volume and over the UROI (the target
    structures dilated by the margin ellipsoid, as in the registration);
  * volume overlap: DSC = 2 |V_D and V_T| / (|V_D| + |V_T|), V_D = the deformed structure
    (mask warp: trilinear of the 0/1 mask, inside when >= 0.5), V_T = the target structure;
  * contours: the deformed structure is opened (erosion then dilation, r times each, by the
    6-connected cross; outside the volume counts as outside) to remove small islands, and its
    boundary (voxels of the set with a 6-neighbour outside it) is the propagated contour; the
    target surface is the boundary of V_T.  SSD of a contour point = the shortest Euclidean
    distance in mm from it to a target-surface point (voxel centres, spacing per axis);
    reported as mean, standard deviation (population) and 95th percentile (linear
    interpolation between order statistics).

The mask warp is FP64: the trilinear value of the 0/1 mask at x + u(x), inside when >= 0.5.
Whether a voxel is inside is an integer that floating point decides, so a voxel whose FP64 value
lies within KNIFE_EDGE of 0.5 may be decided either way by a correct evaluation in single
precision; such knife-edge voxels are listed with each structure, and ``flips`` lets a caller
take their decision the other way, so that every valid result can be enumerated.  Everything
else is exact integer work or FP64.  Distances are computed as ((dx sx)^2 + (dy sy)^2) +
(dz sz)^2 in FP64 with dx, dy, dz integer voxel offsets and the spacings taken as
single-precision values, then the square root of the minimum.
"""
from __future__ import annotations

import numpy as np

from . import uroi as _uroi
from . import warp as _warp

DEFAULT_SPACING = (1.97, 1.97, 2.5)     # mm along x, y, z (section 2.3)

# Bound on |v32 - v64| for the trilinear value v of a 0/1 mask evaluated in single precision
# from the same float32 field: the fraction of each coordinate is exact or off by one rounding
# (2^-24), and each of the seven linear interpolations of values in [0, 1] adds at most one
# rounding, so |v32 - v64| < 1e-6; the margin is four times that.
KNIFE_EDGE = 4e-6


def _neighbour(m: np.ndarray, axis: int, step: int) -> np.ndarray:
    """m at x + step along `axis` (arrays are (z, y, x)); outside the volume reads 0."""
    out = np.zeros_like(m)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if step > 0:
        src[axis] = slice(step, None)
        dst[axis] = slice(None, -step)
    else:
        src[axis] = slice(None, step)
        dst[axis] = slice(-step, None)
    out[tuple(dst)] = m[tuple(src)]
    return out


def erode(m: np.ndarray) -> np.ndarray:
    """Binary erosion by the 6-connected cross: inside when the voxel and its six face
    neighbours are all inside."""
    m = m.astype(bool)
    out = m.copy()
    for axis in range(3):
        for step in (-1, 1):
            out &= _neighbour(m, axis, step)
    return out


def dilate(m: np.ndarray) -> np.ndarray:
    """Binary dilation by the 6-connected cross."""
    m = m.astype(bool)
    out = m.copy()
    for axis in range(3):
        for step in (-1, 1):
            out |= _neighbour(m, axis, step)
    return out


def opening(m: np.ndarray, radius: int) -> np.ndarray:
    m = m.astype(bool)
    for _ in range(radius):
        m = erode(m)
    for _ in range(radius):
        m = dilate(m)
    return m


def boundary(m: np.ndarray) -> np.ndarray:
    """Voxels of the set with at least one face neighbour outside it."""
    m = m.astype(bool)
    return m & ~erode(m)


def surface_distances(contour: np.ndarray, surface: np.ndarray, spacing=DEFAULT_SPACING) -> np.ndarray:
    """For each contour voxel (x-fastest order), the shortest distance in mm to a voxel of
    `surface`, by brute force over all pairs."""
    p = np.argwhere(contour)[:, ::-1]          # (x, y, z) per point, in x-fastest order
    order = np.lexsort((p[:, 0], p[:, 1], p[:, 2]))
    p = p[order]
    q = np.argwhere(surface)[:, ::-1]
    if len(p) == 0 or len(q) == 0:
        return np.zeros(0)
    s = [np.float64(np.float32(v)) for v in spacing]
    out = np.empty(len(p))
    chunk = max(1, (1 << 22) // len(q))
    for a in range(0, len(p), chunk):
        pp = p[a:a + chunk]
        ex = (pp[:, None, 0] - q[None, :, 0]).astype(np.float64) * s[0]
        ey = (pp[:, None, 1] - q[None, :, 1]).astype(np.float64) * s[1]
        ez = (pp[:, None, 2] - q[None, :, 2]).astype(np.float64) * s[2]
        d2 = ex * ex + ey * ey + ez * ez
        out[a:a + chunk] = np.sqrt(d2.min(axis=1))
    return out


def distance_stats(d: np.ndarray) -> dict:
    if len(d) == 0:
        return {"mean": float("nan"), "sd": float("nan"), "p95": float("nan"), "points": 0}
    return {"mean": float(np.mean(d)), "sd": float(np.std(d)),
            "p95": float(np.percentile(d, 95)), "points": int(len(d))}


def dsc(deformed: np.ndarray, target: np.ndarray) -> dict:
    d = deformed.astype(bool)
    t = target.astype(bool)
    nd, nt, no = int(d.sum()), int(t.sum()), int((d & t).sum())
    return {"deformed": nd, "target": nt, "overlap": no,
            "dsc": 2.0 * no / (nd + nt) if nd + nt else float("nan")}


def rms_cc(a: np.ndarray, b: np.ndarray, region=None) -> dict:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if region is not None:
        a = a[region.astype(bool)]
        b = b[region.astype(bool)]
    if a.size == 0:
        return {"rms_id": float("nan"), "cc": float("nan"), "voxels": 0}
    rms = float(np.sqrt(np.mean((a - b) ** 2)))
    da, db = a - a.mean(), b - b.mean()
    den = np.sqrt(np.sum(da * da) * np.sum(db * db))
    cc = float(np.sum(da * db) / den) if den > 0 else float("nan")
    return {"rms_id": rms, "cc": cc, "voxels": int(a.size)}


def deformed_mask(mask: np.ndarray, u) -> tuple:
    """The structure propagated by the field (FP64 mask warp): the inside decision per voxel and
    the knife-edge voxels (flat x-fastest indices) whose trilinear value lies within KNIFE_EDGE
    of 0.5."""
    u64 = np.ascontiguousarray(u, dtype=np.float32).astype(np.float64)
    v = _warp(np.asarray(mask, dtype=bool).astype(np.float64), u64)
    return v >= 0.5, np.flatnonzero(np.abs(v - 0.5) <= KNIFE_EDGE)


def structure(deformed: np.ndarray, target: np.ndarray, spacing=DEFAULT_SPACING, radius: int = 1) -> dict:
    """Overlap and contour metrics of one deformed structure against its target mask."""
    d = deformed.astype(bool)
    t = target.astype(bool)
    rec = dsc(d, t)
    contour = boundary(opening(d, radius))
    rec["ssd"] = distance_stats(surface_distances(contour, boundary(t), spacing))
    return rec


def evaluate(target, moving, target_masks, moving_masks, u, spacing=DEFAULT_SPACING,
             radius: int = 1, margin=(5, 5, 4), flips=None) -> dict:
    """All section 2.3 metrics of the field u (3, nz, ny, nx) registering moving to target.
    flips: optional, one sequence per structure of knife-edge voxels (flat indices) decided the
    other way."""
    u32 = np.ascontiguousarray(u, dtype=np.float32)
    deformed = _warp(moving, u32.astype(np.float64))
    out = {"whole": rms_cc(deformed, target)}
    k = len(target_masks)
    if k:
        region = _uroi(target_masks, margin)
        out["uroi"] = rms_cc(deformed, target, region)
    out["structures"] = []
    for i in range(k):
        d, knife = deformed_mask(moving_masks[i], u32)
        if flips is not None and len(flips[i]):
            f = np.asarray(flips[i], dtype=np.int64)
            if not np.isin(f, knife).all():
                raise ValueError("only knife-edge voxels may be decided the other way")
            d = d.copy()
            d.flat[f] = ~d.flat[f]
        rec = structure(d, target_masks[i], spacing, radius)
        rec["knife_edge"] = [int(x) for x in knife]
        out["structures"].append(rec)
    return out
