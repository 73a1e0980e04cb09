"""FP64 CPU oracle of contour-guided demons registration (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The registration library
never calls it, and it imports nothing from the library.

Arrays follow the library's layout: volumes (nz, ny, nx) x-fastest; displacement
fields (3, nz, ny, nx) with components (x, y, z) in voxel units.  Inputs are converted
to float64 here; outputs are float64.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcgdir_oracle.so")
_lib = None

MAX_STRUCTS = 32
MAX_LEVELS = 8

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class _Params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("iters", ctypes.c_int * MAX_LEVELS),
        ("contour_level_mask", ctypes.c_uint),
        ("sigma_fluid", ctypes.c_double),
        ("sigma_diff", ctypes.c_double),
        ("restrict_sigma", ctypes.c_double),
        ("lambda_", ctypes.c_double * MAX_STRUCTS),
        ("sign", ctypes.c_int * MAX_STRUCTS),
        ("c0", ctypes.c_double),
        ("stop_mode", ctypes.c_int),
        ("stop_eps", ctypes.c_double),
        ("stop_window", ctypes.c_int),
        ("norm_range", ctypes.c_double),
        ("uroi_radius", ctypes.c_int * 3),
        ("spacing", ctypes.c_double * 3),
    ]


@dataclasses.dataclass
class Params:
    """Registration parameters (section 2.2): defaults follow the paper where it gives one."""
    levels: int = 1
    iters: Sequence[int] = (100,)
    contour_level_mask: int = 1
    sigma_fluid: float = 1.0
    sigma_diff: float = 1.0
    restrict_sigma: float = 1.0
    lambdas: Optional[Sequence[float]] = None   # default 1e-3 for every structure
    signs: Optional[Sequence[int]] = None       # default +1
    c0: float = 1000.0
    stop_mode: int = 0
    stop_eps: float = 1e-4
    stop_window: int = 10
    norm_range: float = 2500.0
    uroi_radius: Sequence[int] = (5, 5, 4)
    spacing: Optional[Sequence[float]] = None   # finest voxel size (x, y, z); None = voxel units

    def to_c(self, k: int) -> _Params:
        p = _Params()
        p.levels = int(self.levels)
        for i, v in enumerate(self.iters):
            p.iters[i] = int(v)
        p.contour_level_mask = int(self.contour_level_mask)
        p.sigma_fluid = float(self.sigma_fluid)
        p.sigma_diff = float(self.sigma_diff)
        p.restrict_sigma = float(self.restrict_sigma)
        lam = self.lambdas if self.lambdas is not None else [1e-3] * k
        sg = self.signs if self.signs is not None else [1] * k
        for i in range(k):
            p.lambda_[i] = float(lam[i])
            p.sign[i] = int(sg[i])
        p.c0 = float(self.c0)
        p.stop_mode = int(self.stop_mode)
        p.stop_eps = float(self.stop_eps)
        p.stop_window = int(self.stop_window)
        p.norm_range = float(self.norm_range)
        for i in range(3):
            p.uroi_radius[i] = int(self.uroi_radius[i])
            p.spacing[i] = float(self.spacing[i]) if self.spacing is not None else 0.0
        return p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.orc_sample.restype = ctypes.c_double
        _lib.orc_eq7.restype = ctypes.c_double
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _ptr(a):
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    return a.ctypes.data_as(_u8p)


def _dims(vol):
    nz, ny, nx = vol.shape[-3:]
    return nx, ny, nz


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments (rc=%d)" % (what, rc))


def gauss_weights(sigma: float) -> np.ndarray:
    R = lib().orc_gauss_radius(ctypes.c_double(sigma))
    w = np.zeros(2 * R + 1)
    lib().orc_gauss_weights(ctypes.c_double(sigma), _ptr(w))
    return w


def smooth(f, sigma: float) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    _check(lib().orc_smooth(_ptr(f), *_dims(f), ctypes.c_double(sigma), _ptr(out)), "smooth")
    return out


def smooth_axes(f, sigmas) -> np.ndarray:
    """Separable Gaussian with its own sigma (voxels) along x, y, z."""
    f = _f64(f)
    out = np.empty_like(f)
    s = _f64(np.asarray(sigmas, float))
    _check(lib().orc_smooth_axes(_ptr(f), *_dims(f), _ptr(s), _ptr(out)), "smooth_axes")
    return out


def _h(spacing):
    return _f64(np.asarray(spacing, float)) if spacing is not None else None


def sample(f, px, py, pz) -> float:
    f = _f64(f)
    return lib().orc_sample(_ptr(f), *_dims(f), ctypes.c_double(px), ctypes.c_double(py),
                            ctypes.c_double(pz))


def warp(f, u) -> np.ndarray:
    f = _f64(f)
    u = _f64(u)
    out = np.empty_like(f)
    _check(lib().orc_warp(_ptr(f), *_dims(f), _ptr(u), _ptr(out)), "warp")
    return out


def warp_mask(m, u) -> np.ndarray:
    m = _u8(m)
    u = _f64(u)
    out = np.empty_like(m)
    _check(lib().orc_warp_mask(_ptr(m), *_dims(m), _ptr(u), _ptr(out)), "warp_mask")
    return out


def gradient(f, spacing=None) -> np.ndarray:
    """Central differences (clamped), divided by the voxel size (x, y, z) when given."""
    f = _f64(f)
    g = np.empty((3,) + f.shape)
    h = _h(spacing)
    _check(lib().orc_gradient_h(_ptr(f), *_dims(f), _ptr(h) if h is not None else None, _ptr(g)), "gradient")
    return g


def compose(u, du) -> np.ndarray:
    u = _f64(u)
    du = _f64(du)
    out = np.empty_like(u)
    _check(lib().orc_compose(_ptr(u), _ptr(du), *_dims(u), _ptr(out)), "compose")
    return out


def restrict(f, sigma: float = 1.0) -> np.ndarray:
    f = _f64(f)
    nx, ny, nz = _dims(f)
    out = np.empty(((nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2))
    _check(lib().orc_restrict(_ptr(f), nx, ny, nz, ctypes.c_double(sigma), _ptr(out)), "restrict")
    return out


def decimate_masks(masks) -> np.ndarray:
    """Masks (k, nz, ny, nx) at the next coarser pyramid level (contour terms below the
    finest level): inside where the fine voxel at the even indices is inside."""
    masks = _u8(masks)
    k = masks.shape[0]
    nx, ny, nz = _dims(masks)
    out = np.empty((k, (nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2), np.uint8)
    _check(lib().orc_decimate_masks(_ptr(masks), k, nx, ny, nz, _ptr(out)), "decimate_masks")
    return out


def prolong(uc, fine_dims) -> np.ndarray:
    uc = _f64(uc)
    fnx, fny, fnz = fine_dims
    out = np.empty((3, fnz, fny, fnx))
    _check(lib().orc_prolong(_ptr(uc), *_dims(uc), fnx, fny, fnz, _ptr(out)), "prolong")
    return out


def uroi(masks, radius=(5, 5, 4)) -> np.ndarray:
    masks = _u8(masks)
    k = masks.shape[0]
    out = np.empty(masks.shape[1:], np.uint8)
    r = (ctypes.c_int * 3)(*radius)
    _check(lib().orc_uroi(_ptr(masks), k, *_dims(masks), r, _ptr(out)), "uroi")
    return out


def auto_sign(T0, mask, radius=(5, 5, 4)) -> int:
    T0 = _f64(T0)
    mask = _u8(mask)
    r = (ctypes.c_int * 3)(*radius)
    return int(lib().orc_auto_sign(_ptr(T0), _ptr(mask), *_dims(T0), r))


def modified_image(F, mask, s: int, c0: float = 1000.0) -> np.ndarray:
    F = _f64(F)
    mask = _u8(mask)
    out = np.empty_like(F)
    _check(lib().orc_modified_image(_ptr(F), _ptr(mask), int(s), ctypes.c_double(c0),
                                    ctypes.c_size_t(F.size), _ptr(out)), "modified_image")
    return out


def eq7(a0, d, lambdas, a, di) -> float:
    k = len(lambdas)
    lam = _f64(np.asarray(lambdas, float).reshape(-1) if k else np.zeros(1))
    aa = _f64(np.asarray(a, float).reshape(-1) if k else np.zeros(1))
    dd = _f64(np.asarray(di, float).reshape(-1) if k else np.zeros(1))
    return lib().orc_eq7(ctypes.c_double(a0), ctypes.c_double(d), k, _ptr(lam), _ptr(aa), _ptr(dd))


def _ptr_array(arrs):
    t = (_dp * max(len(arrs), 1))()
    for i, a in enumerate(arrs):
        t[i] = _ptr(a)
    return t


def force(wI0, T0, wIp, Tp, lambdas, spacing=None) -> np.ndarray:
    wI0 = _f64(wI0)
    T0 = _f64(T0)
    wIp = [_f64(a) for a in wIp]
    Tp = [_f64(a) for a in Tp]
    k = len(wIp)
    lam = _f64(np.asarray(lambdas, float).reshape(-1) if k else np.zeros(1))
    du = np.empty((3,) + wI0.shape)
    h = _h(spacing)
    _check(lib().orc_force_h(_ptr(wI0), _ptr(T0), k, _ptr_array(wIp), _ptr_array(Tp), _ptr(lam),
                             *_dims(wI0), _ptr(h) if h is not None else None, _ptr(du)), "force")
    return du


def step(I0, T0, Iplus, Tplus, lambdas, sigma_f, sigma_d, u, uroi_mask=None,
         norm_range=2500.0, spacing=None):
    """One iteration from u (not modified); returns (u_next, delta or None)."""
    I0 = _f64(I0)
    T0 = _f64(T0)
    Ip = [_f64(a) for a in Iplus]
    Tp = [_f64(a) for a in Tplus]
    k = len(Ip)
    lam = _f64(np.asarray(lambdas, float).reshape(-1) if k else np.zeros(1))
    un = _f64(u).copy()
    delta = ctypes.c_double(0.0)
    ur = _u8(uroi_mask) if uroi_mask is not None else None
    h = _h(spacing)
    _check(lib().orc_step(_ptr(I0), _ptr(T0), *_dims(I0), k, _ptr_array(Ip), _ptr_array(Tp),
                          _ptr(lam), ctypes.c_double(sigma_f), ctypes.c_double(sigma_d),
                          _ptr(h) if h is not None else None,
                          _ptr(ur) if ur is not None else None, ctypes.c_double(norm_range),
                          _ptr(un), ctypes.byref(delta) if ur is not None else None), "step")
    return un, (delta.value if ur is not None else None)


def register(target, moving, target_masks, moving_masks, params: Params, initial_u=None,
             want_delta: bool = False):
    """Algorithm A.  Returns (u, delta_history or None, finest-level iterations run)."""
    T = _f64(target)
    I = _f64(moving)
    tm = _u8(target_masks)
    mm = _u8(moving_masks)
    k = tm.shape[0] if tm.ndim == 4 else 0
    if k == 0:
        tm = np.zeros((1,) + T.shape, np.uint8)
        mm = tm
    u = np.empty((3,) + T.shape)
    hist = np.zeros(max(int(params.iters[0]), 1)) if want_delta else None
    done = ctypes.c_int(0)
    iu = _f64(initial_u) if initial_u is not None else None
    cp = params.to_c(k)
    _check(lib().orc_register(_ptr(T), _ptr(I), *_dims(T), k, _ptr(tm), _ptr(mm), ctypes.byref(cp),
                              _ptr(iu) if iu is not None else None, _ptr(u),
                              _ptr(hist) if hist is not None else None, ctypes.byref(done)),
           "register")
    if hist is not None:
        hist = hist[: done.value]
    return u, hist, done.value


def params_for(pair, **over) -> Params:
    """Parameters of a synthetic pair (sigma of both smoothings, levels, iterations)."""
    p = Params(levels=pair.levels, iters=tuple(pair.iters), sigma_fluid=pair.sigma,
               sigma_diff=pair.sigma, lambdas=[1e-3] * pair.k, signs=list(pair.signs))
    for key, v in over.items():
        setattr(p, key, v)
    return p
