"""Python binding of libcgdir (include/cgdir.h): argument marshalling only.

Every step of the registration runs in the library's HIP kernels; PyTorch only supplies
device memory (tensor ``data_ptr``) and the stream.  The library is loaded from
``paper_1301_0970_amd/lib/libcgdir.so``; if it is missing, importing this module
raises (there is no fallback implementation).

Names mirror the C entry points: ``create``, ``destroy``, ``register``, ``warp``,
``register_batch``, ``submit``, ``poll``, ``cancel``, ``wait``, ``footprint``,
``strerror``, ``params_default``, ``kernel_stats``, ``evaluate``, ``tuning_export``,
``tuning_import``.  :class:`Context` wraps them for
torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libcgdir.so")

MAX_STRUCTS = 8
MAX_LEVELS = 6
KEEP_FINISHED = 4096   # served requests whose final status a context keeps

OK = 0
E_INVAL, E_NOMEM, E_HIP, E_BUSY, E_NOTFOUND, E_CANCELLED, E_NONFINITE, E_UNIMPL, E_TIMEOUT, E_SCRATCH = (
    -1, -2, -3, -4, -5, -6, -7, -8, -9, -10)
STATIC_SCRATCH_BYTES = 64 << 20   # device memory of cgdir_register_static, per device
HOST, DEVICE = 0, 1
WARP_LINEAR, WARP_MASK = 0, 1
QUEUED, RUNNING, DONE, FAILED, CANCELLED = 0, 1, 2, 3, 4
CTX_PROFILE = 1


class CgdirError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))
        self.code = code


class ctx_desc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("pool", ctypes.c_void_p),
                ("pool_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int), ("flags", ctypes.c_int)]


class volume(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("where", ctypes.c_int)]


class masks(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("planes", ctypes.POINTER(ctypes.c_void_p)),
                ("where", ctypes.c_int)]


class params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("iters", ctypes.c_int * MAX_LEVELS),
        ("contour_level_mask", ctypes.c_uint),
        ("sigma_fluid", ctypes.c_float),
        ("sigma_diff", ctypes.c_float),
        ("restrict_sigma", ctypes.c_float),
        ("lambda_", ctypes.c_float * MAX_STRUCTS),
        ("sign", ctypes.c_int * MAX_STRUCTS),
        ("intensity_offset", ctypes.c_float),
        ("stop_mode", ctypes.c_int),
        ("stop_eps", ctypes.c_float),
        ("stop_window", ctypes.c_int),
        ("norm_range", ctypes.c_float),
        ("uroi_margin", ctypes.c_int * 3),
        ("initial_dvf", ctypes.c_void_p),
        ("initial_dvf_where", ctypes.c_int),
        ("delta_hist", ctypes.POINTER(ctypes.c_double)),
        ("iters_done", ctypes.POINTER(ctypes.c_int)),
        ("spacing", ctypes.c_float * 3),
    ]


class request(ctypes.Structure):
    _fields_ = [("target", volume), ("moving", volume), ("target_masks", masks),
                ("moving_masks", masks), ("params", params), ("dvf_out", ctypes.c_void_p),
                ("dvf_where", ctypes.c_int)]


class status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("error", ctypes.c_int), ("level", ctypes.c_int),
                ("iter", ctypes.c_int), ("last_delta", ctypes.c_double),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("voxels", ctypes.c_double)]


SYMBOLS = ["cgdir_params_default", "cgdir_create", "cgdir_destroy", "cgdir_register",
           "cgdir_warp", "cgdir_register_batch", "cgdir_submit", "cgdir_poll", "cgdir_cancel",
           "cgdir_wait", "cgdir_footprint", "cgdir_strerror", "cgdir_kernel_stats",
           "cgdir_eval_params_default", "cgdir_evaluate", "cgdir_tuning_export", "cgdir_tuning_import",
           "cgdir_register_static"]


class eval_params(ctypes.Structure):
    _fields_ = [("spacing", ctypes.c_float * 3), ("opening_radius", ctypes.c_int),
                ("uroi_margin", ctypes.c_int * 3)]


_S = MAX_STRUCTS


class eval_result(ctypes.Structure):
    _fields_ = [("rms_id", ctypes.c_double), ("cc", ctypes.c_double),
                ("rms_id_uroi", ctypes.c_double), ("cc_uroi", ctypes.c_double),
                ("voxels", ctypes.c_int64), ("uroi_voxels", ctypes.c_int64), ("k", ctypes.c_int),
                ("deformed_voxels", ctypes.c_int64 * _S), ("target_voxels", ctypes.c_int64 * _S),
                ("overlap_voxels", ctypes.c_int64 * _S), ("dsc", ctypes.c_double * _S),
                ("contour_points", ctypes.c_int64 * _S), ("surface_points", ctypes.c_int64 * _S),
                ("ssd_mean", ctypes.c_double * _S), ("ssd_sd", ctypes.c_double * _S),
                ("ssd_p95", ctypes.c_double * _S)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcgdir.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one the library binds
    # to.  Loaded the other way round, the process ends up with two HIP runtimes and the
    # library's cannot open the device that torch's already holds.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.cgdir_params_default.argtypes = [P(params)]
    lib.cgdir_params_default.restype = None
    lib.cgdir_create.argtypes = [P(ctypes.c_void_p), P(ctx_desc)]
    lib.cgdir_destroy.argtypes = [ctypes.c_void_p]
    lib.cgdir_register.argtypes = [ctypes.c_void_p, P(volume), P(volume), P(masks), P(masks),
                                   P(params), ctypes.c_void_p, ctypes.c_int]
    lib.cgdir_warp.argtypes = [ctypes.c_void_p, P(volume), ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_void_p]
    lib.cgdir_register_batch.argtypes = [ctypes.c_void_p, ctypes.c_int, P(request), P(ctypes.c_int)]
    lib.cgdir_submit.argtypes = [ctypes.c_void_p, P(request), P(ctypes.c_uint64)]
    lib.cgdir_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(status)]
    lib.cgdir_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.cgdir_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64]
    lib.cgdir_footprint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    P(params)]
    lib.cgdir_footprint.restype = ctypes.c_size_t
    lib.cgdir_strerror.argtypes = [ctypes.c_int]
    lib.cgdir_strerror.restype = ctypes.c_char_p
    lib.cgdir_kernel_stats.argtypes = [ctypes.c_void_p, P(kernel_stat), ctypes.c_int, ctypes.c_int]
    lib.cgdir_eval_params_default.argtypes = [P(eval_params)]
    lib.cgdir_eval_params_default.restype = None
    lib.cgdir_evaluate.argtypes = [ctypes.c_void_p, P(volume), P(volume), P(masks), P(masks),
                                   ctypes.c_void_p, ctypes.c_int, P(eval_params), P(eval_result)]
    lib.cgdir_tuning_export.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_size_t)]
    lib.cgdir_tuning_import.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    lib.cgdir_register_static.argtypes = [ctypes.c_void_p, P(volume), P(volume), P(masks), P(masks),
                                          P(params), ctypes.c_void_p]
    for name in SYMBOLS:
        if name not in ("cgdir_params_default", "cgdir_footprint", "cgdir_strerror",
                        "cgdir_eval_params_default"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


LIB = _load()


# ----------------------------------------------------------------------------- raw calls

def strerror(code: int) -> str:
    return LIB.cgdir_strerror(int(code)).decode()


def params_default() -> params:
    p = params()
    LIB.cgdir_params_default(ctypes.byref(p))
    return p


def footprint(nx: int, ny: int, nz: int, k: int, prm: Optional[params] = None) -> int:
    return int(LIB.cgdir_footprint(nx, ny, nz, k, ctypes.byref(prm) if prm is not None else None))


def create(desc: ctx_desc) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = LIB.cgdir_create(ctypes.byref(h), ctypes.byref(desc))
    if rc != OK:
        raise CgdirError(rc, "cgdir_create")
    return h


def destroy(h) -> int:
    return LIB.cgdir_destroy(h)


def register(h, target: volume, moving: volume, target_masks: Optional[masks],
             moving_masks: Optional[masks], prm: params, dvf_out: int, dvf_where: int) -> int:
    return LIB.cgdir_register(h, ctypes.byref(target), ctypes.byref(moving),
                              ctypes.byref(target_masks) if target_masks is not None else None,
                              ctypes.byref(moving_masks) if moving_masks is not None else None,
                              ctypes.byref(prm), ctypes.c_void_p(dvf_out), dvf_where)


def register_static(h, target: volume, moving: volume, target_masks: Optional[masks],
                    moving_masks: Optional[masks], prm: params, dvf_out: int) -> int:
    return LIB.cgdir_register_static(h, ctypes.byref(target), ctypes.byref(moving),
                                     ctypes.byref(target_masks) if target_masks is not None else None,
                                     ctypes.byref(moving_masks) if moving_masks is not None else None,
                                     ctypes.byref(prm), ctypes.c_void_p(dvf_out))


def warp(h, src: volume, dvf: int, mode: int, out: int) -> int:
    return LIB.cgdir_warp(h, ctypes.byref(src), ctypes.c_void_p(dvf), mode, ctypes.c_void_p(out))


def register_batch(h, reqs: Sequence[request], st=None) -> int:
    arr = (request * len(reqs))(*reqs)
    return LIB.cgdir_register_batch(h, len(reqs), arr, st)


def submit(h, req: request) -> (int, int):
    t = ctypes.c_uint64(0)
    rc = LIB.cgdir_submit(h, ctypes.byref(req), ctypes.byref(t))
    return rc, t.value


def poll(h, ticket: int) -> (int, status):
    st = status()
    rc = LIB.cgdir_poll(h, ctypes.c_uint64(ticket), ctypes.byref(st))
    return rc, st


def cancel(h, ticket: int) -> int:
    return LIB.cgdir_cancel(h, ctypes.c_uint64(ticket))


def wait(h, ticket: int, timeout_ns: int = -1) -> int:
    return LIB.cgdir_wait(h, ctypes.c_uint64(ticket), ctypes.c_int64(timeout_ns))


def tuning_export(h) -> str:
    n = ctypes.c_size_t(0)
    _check(LIB.cgdir_tuning_export(h, None, 0, ctypes.byref(n)), "cgdir_tuning_export")
    buf = ctypes.create_string_buffer(n.value)
    _check(LIB.cgdir_tuning_export(h, buf, n.value, ctypes.byref(n)), "cgdir_tuning_export")
    return buf.value.decode()


def tuning_import(h, text: str) -> int:
    return LIB.cgdir_tuning_import(h, text.encode())


def kernel_stats(h, reset: bool = False) -> List[dict]:
    arr = (kernel_stat * 32)()
    n = LIB.cgdir_kernel_stats(h, arr, 32, 1 if reset else 0)
    if n < 0:
        raise CgdirError(n, "cgdir_kernel_stats")
    return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                 voxels=arr[i].voxels) for i in range(n)]


# ----------------------------------------------------------------------------- torch glue

def _check(rc, what):
    if rc != OK:
        raise CgdirError(rc, what)


def make_params(levels=1, iters=(100,), sigma_fluid=1.0, sigma_diff=1.0, restrict_sigma=1.0,
                lambdas=None, signs=None, c0=1000.0, stop_mode=0, stop_eps=1e-4, stop_window=10,
                norm_range=2500.0, uroi_margin=(5, 5, 4), contour_level_mask=1, spacing=None) -> params:
    """Library parameters; spacing = finest voxel size (x, y, z) for physical units, None for
    voxel units (then sigma_fluid and sigma_diff are in voxels)."""
    p = params_default()
    p.levels = int(levels)
    for i, v in enumerate(iters):
        p.iters[i] = int(v)
    p.sigma_fluid = float(sigma_fluid)
    p.sigma_diff = float(sigma_diff)
    p.restrict_sigma = float(restrict_sigma)
    if lambdas is not None:
        for i, v in enumerate(lambdas):
            p.lambda_[i] = float(v)
    if signs is not None:
        for i, v in enumerate(signs):
            p.sign[i] = int(v)
    p.intensity_offset = float(c0)
    p.stop_mode = int(stop_mode)
    p.stop_eps = float(stop_eps)
    p.stop_window = int(stop_window)
    p.norm_range = float(norm_range)
    for i in range(3):
        p.uroi_margin[i] = int(uroi_margin[i])
    p.contour_level_mask = int(contour_level_mask)
    if spacing is not None:
        p.spacing[:] = [float(v) for v in spacing]
    return p


class Context:
    """A libcgdir context on one GPU, with a pool carved from one torch tensor.

    Volumes are torch tensors shaped (nz, ny, nx) (float32 images, uint8 masks) and
    fields (3, nz, ny, nx) float32, on ``cuda:device`` (device-resident) or on the CPU
    (host; the library copies them)."""

    def __init__(self, pool_bytes: int, device: int = 0, max_slots: int = 4, profile=False,
                 stream=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", device)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        # The library orders its work on its own stream only.  Every call first makes that
        # stream wait for the caller's current stream (_order), so that device inputs that
        # torch is still computing are complete before the library reads them.  (torch's
        # default stream has the handle 0, which the library would replace by a stream of its
        # own, so the context gets a dedicated stream of default priority instead.)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        d = ctx_desc(device=device, stream=self.stream.cuda_stream, pool=self.pool.data_ptr(),
                     pool_bytes=int(pool_bytes), max_slots=int(max_slots),
                     flags=CTX_PROFILE if profile else 0)
        self.handle = create(d)
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None) is not None:
            destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- marshalling
    def _order(self):
        cur = self._torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _where(self, t):
        return DEVICE if t.is_cuda else HOST

    def _plain(self, t, dtype, what):
        """The library reads raw, densely packed memory: dtype and layout must match."""
        if t.dtype != dtype:
            raise ValueError("%s must be %s, not %s" % (what, dtype, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous (x fastest)" % what)
        return t

    def _field(self, t, like, what):
        """A field of three float32 planes of like's voxels (the library reads or writes
        3 * like.numel() floats; the volumes themselves it checks)."""
        self._plain(t, self._torch.float32, what)
        if t.numel() < 3 * like.numel():
            raise ValueError("%s holds %d floats, fewer than 3 x %d" % (what, t.numel(), like.numel()))
        return t

    def volume(self, t) -> volume:
        self._plain(t, self._torch.float32, "a volume")
        nz, ny, nx = t.shape
        return volume(t.data_ptr(), nx, ny, nz, self._where(t))

    def masks(self, m, keep: list) -> masks:
        if m is None or m.shape[0] == 0:
            return masks(0, None, DEVICE)
        self._plain(m, self._torch.uint8, "masks")
        k = m.shape[0]
        ptrs = (ctypes.c_void_p * k)(*[m[i].data_ptr() for i in range(k)])
        keep.append(ptrs)
        return masks(k, ptrs, self._where(m))

    def request(self, target, moving, target_masks, moving_masks, prm: params, out, keep) -> request:
        self._field(out, target, "the output field")
        return request(self.volume(target), self.volume(moving), self.masks(target_masks, keep),
                       self.masks(moving_masks, keep), prm, out.data_ptr(), self._where(out))

    # -- calls
    def register(self, target, moving, target_masks=None, moving_masks=None, prm=None, out=None,
                 initial=None, delta=False):
        """Blocking registration; returns the field (3, nz, ny, nx) and, with delta=True,
        (field, delta history, iterations run at the finest level)."""
        torch = self._torch
        prm = params.from_buffer_copy(prm) if prm is not None else params_default()
        if out is None:
            out = torch.empty((3,) + tuple(target.shape), dtype=torch.float32, device=target.device)
        self._field(out, target, "the output field")
        keep = []
        hist = None
        done = ctypes.c_int(0)
        if initial is not None:
            self._field(initial, target, "the initial field")
            prm.initial_dvf = initial.data_ptr()
            prm.initial_dvf_where = self._where(initial)
        if delta:
            hist = (ctypes.c_double * max(int(prm.iters[0]), 1))()
            prm.delta_hist = hist
        prm.iters_done = ctypes.pointer(done)
        tm = self.masks(target_masks, keep)
        mm = self.masks(moving_masks, keep)
        tv, mv = self.volume(target), self.volume(moving)
        self._order()
        rc = register(self.handle, tv, mv, tm, mm, prm, out.data_ptr(), self._where(out))
        _check(rc, "cgdir_register")
        if delta:
            return out, [hist[i] for i in range(done.value)], done.value
        return out

    def register_static(self, target, moving, target_masks=None, moving_masks=None, prm=None, out=None,
                        initial=None):
        """cgdir_register_static: the registration on device tensors, its buffers in the
        library's static device scratch instead of the pool (nothing is allocated)."""
        torch = self._torch
        prm = params.from_buffer_copy(prm) if prm is not None else params_default()
        if out is None:
            out = torch.empty((3,) + tuple(target.shape), dtype=torch.float32, device=target.device)
        self._field(out, target, "the output field")
        keep = []
        if initial is not None:
            self._field(initial, target, "the initial field")
            prm.initial_dvf = initial.data_ptr()
            prm.initial_dvf_where = self._where(initial)
        tm = self.masks(target_masks, keep)
        mm = self.masks(moving_masks, keep)
        tv, mv = self.volume(target), self.volume(moving)
        self._order()
        _check(register_static(self.handle, tv, mv, tm, mm, prm, out.data_ptr()), "cgdir_register_static")
        return out

    def warp(self, src, dvf, mode=WARP_LINEAR, out=None):
        torch = self._torch
        if out is None:
            out = torch.empty_like(src)
        sv = self.volume(src) if mode == WARP_LINEAR else self._mask_volume(src)
        self._field(dvf, src, "the field")
        self._plain(out, src.dtype, "the output")
        self._order()
        _check(warp(self.handle, sv, dvf.data_ptr(), mode, out.data_ptr()), "cgdir_warp")
        return out

    def _mask_volume(self, t) -> volume:
        self._plain(t, self._torch.uint8, "a mask")
        nz, ny, nx = t.shape
        return volume(t.data_ptr(), nx, ny, nz, self._where(t))

    def evaluate(self, target, moving, target_masks, moving_masks, dvf, spacing=None,
                 opening_radius=None, uroi_margin=None) -> dict:
        """Section 2.3 metrics of the field dvf registering moving to target (RMS-ID, CC,
        DSC, SSD statistics of the propagated contours), computed on the GPU."""
        ep = eval_params()
        LIB.cgdir_eval_params_default(ctypes.byref(ep))
        if spacing is not None:
            ep.spacing[:] = [float(v) for v in spacing]
        if opening_radius is not None:
            ep.opening_radius = int(opening_radius)
        if uroi_margin is not None:
            ep.uroi_margin[:] = [int(v) for v in uroi_margin]
        keep = []
        res = eval_result()
        tv, mv = self.volume(target), self.volume(moving)
        tm, mm = self.masks(target_masks, keep), self.masks(moving_masks, keep)
        self._field(dvf, target, "the field")
        self._order()
        rc = LIB.cgdir_evaluate(self.handle, ctypes.byref(tv), ctypes.byref(mv), ctypes.byref(tm), ctypes.byref(mm),
                                dvf.data_ptr(), self._where(dvf), ctypes.byref(ep), ctypes.byref(res))
        _check(rc, "cgdir_evaluate")
        out = {"whole": {"rms_id": res.rms_id, "cc": res.cc, "voxels": res.voxels}, "structures": []}
        if res.k:
            out["uroi"] = {"rms_id": res.rms_id_uroi, "cc": res.cc_uroi, "voxels": res.uroi_voxels}
        for i in range(res.k):
            out["structures"].append({
                "deformed": res.deformed_voxels[i], "target": res.target_voxels[i],
                "overlap": res.overlap_voxels[i], "dsc": res.dsc[i],
                "ssd": {"mean": res.ssd_mean[i], "sd": res.ssd_sd[i], "p95": res.ssd_p95[i],
                        "points": res.contour_points[i]},
                "surface_points": res.surface_points[i]})
        return out

    def register_batch(self, items, prms, outs):
        keep = []
        reqs = [self.request(t, m, tm, mm, p, o, keep) for (t, m, tm, mm), p, o in zip(items, prms, outs)]
        st = (ctypes.c_int * len(reqs))()
        self._order()
        rc = register_batch(self.handle, reqs, st)
        return rc, [st[i] for i in range(len(reqs))]

    def submit(self, target, moving, target_masks, moving_masks, prm, out):
        keep = []
        req = self.request(target, moving, target_masks, moving_masks, prm, out, keep)
        self._order()
        rc, t = submit(self.handle, req)
        _check(rc, "cgdir_submit")
        self._keep[t] = (keep, target, moving, target_masks, moving_masks, out)
        if len(self._keep) > KEEP_FINISHED:   # tickets never waited on: drop finished ones
            for old in list(self._keep)[: len(self._keep) - KEEP_FINISHED // 2]:
                prc, st = poll(self.handle, old)
                if prc == E_NOTFOUND or (prc == OK and st.state in (DONE, FAILED, CANCELLED)):
                    self._keep.pop(old, None)
        return t

    def poll(self, ticket):
        rc, st = poll(self.handle, ticket)
        _check(rc, "cgdir_poll")
        if st.state in (DONE, FAILED, CANCELLED):   # the library is done with the tensors
            self._keep.pop(ticket, None)
        return st

    def wait(self, ticket, timeout_ns=-1):
        rc = wait(self.handle, ticket, timeout_ns)
        if rc != E_TIMEOUT:
            self._keep.pop(ticket, None)
        return rc

    def cancel(self, ticket):
        return cancel(self.handle, ticket)

    def kernel_stats(self, reset=False):
        return kernel_stats(self.handle, reset)

    def tuning_export(self) -> str:
        """The settled tile-shape groups as text (see cgdir_tuning_export)."""
        return tuning_export(self.handle)

    def tuning_import(self, text: str):
        """Settle tile-shape groups from text an earlier context exported."""
        _check(tuning_import(self.handle, text), "cgdir_tuning_import")


def params_for_pair(pair, **over) -> params:
    """Library parameters of a synthetic pair (sigma of both smoothings, levels, iterations)."""
    kw = dict(levels=pair.levels, iters=pair.iters, sigma_fluid=pair.sigma, sigma_diff=pair.sigma,
              lambdas=[1e-3] * pair.k, signs=list(pair.signs))
    kw.update(over)
    return make_params(**kw)
