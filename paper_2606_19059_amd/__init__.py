"""MI355X spectral Ewald summation of the triply periodic Stokeslet sum.

Thin ctypes binding over the C ABI of ``include/ewald.h`` (``libewald.so``, built by
``paper_2606_19059_amd.build``).  It only marshals arguments: every step of the
evaluation runs in the library's HIP kernels.  PyTorch provides device memory and
streams.  If the library is missing, every entry point raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libewald.so")

EWALD_OK = 0
EWALD_EINVAL = -1
EWALD_ENOMEM = -2
EWALD_EHIP = -3
EWALD_EUNSUPPORTED = -4
EWALD_FP64 = 0
EWALD_FP32_BULK = 1
EWALD_FLAG_P2P_FP64_ACC = 1 << 8
EWALD_FLAG_STAGE_TIMERS = 1 << 9
EWALD_FLAG_WINDOW_KB = 1 << 10
EWALD_FLAG_DETERMINISTIC = 1 << 11
EWALD_FLAG_STRESSLET = 1 << 12
EWALD_FLAG_CHECK_INPUTS = 1 << 13

NOALLOC_MAX_WORKSPACE = 64 << 20  # EWALD_NOALLOC_MAX_WORKSPACE
MAX_BATCH = 64  # EWALD_MAX_BATCH

STAGES = ("sort", "p2p", "p2g", "fgc", "g2p", "total")

# every function declared in include/ewald.h
EXPORTS = (
    "ewald_plan_create",
    "ewald_resolve",
    "ewald_plan_get_info",
    "ewald_plan_destroy",
    "ewald_workspace_bytes",
    "ewald_eval",
    "ewald_eval_batch",
    "ewald_workspace_bytes_batch",
    "ewald_eval_noalloc",
    "ewald_eval_overlap",
    "ewald_eval_parts",
    "ewald_eval_combined",
    "ewald_eval_combined_parts",
    "ewald_spread",
    "ewald_far_grid",
    "ewald_count_pairs",
    "ewald_stage_ms",
    "ewald_debug_fail_next",
    "ewald_last_error",
    "ewald_version",
)


class EwaldError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ewald error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("xi", ctypes.c_double),
        ("r_c", ctypes.c_double),
        ("grid", ctypes.c_int32 * 3),
        ("P", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("n_max", ctypes.c_int64),
        ("window_shape", ctypes.c_double),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("params", Params),
        ("h", ctypes.c_double * 3),
        ("err_near", ctypes.c_double),
        ("err_far", ctypes.c_double),
        ("err_window", ctypes.c_double),
        ("tile", ctypes.c_int32),
        ("n_tiles", ctypes.c_int32 * 3),
        ("stencil", ctypes.c_int32 * 3),
        ("fourier_fp64", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64),
        ("predicted_ms", ctypes.c_double),
        ("self_coef", ctypes.c_double),
        ("grid_bytes", ctypes.c_int64),
    ]


_lib = None


def load(path: str | None = None):
    """Load libewald.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            "HIP library %s is missing: build it with `python -m paper_2606_19059_amd.build` "
            "(there is no CPU fallback)" % p
        )
    lib = ctypes.CDLL(p)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.ewald_plan_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(vp)]
    lib.ewald_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.ewald_resolve.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(PlanInfo)]
    lib.ewald_plan_destroy.argtypes = [vp]
    lib.ewald_workspace_bytes.argtypes = [vp, i64]
    lib.ewald_workspace_bytes.restype = i64
    for name in ("ewald_eval", "ewald_eval_parts"):
        getattr(lib, name).argtypes = [vp, i64, vp, vp, vp] + ([vp] if name == "ewald_eval_parts" else []) + [vp, i64, vp]
    lib.ewald_eval_noalloc.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.ewald_eval_batch.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, vp, i64, vp]
    lib.ewald_workspace_bytes_batch.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.ewald_workspace_bytes_batch.restype = i64
    lib.ewald_eval_overlap.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp]
    for name in ("ewald_eval_combined", "ewald_eval_combined_parts"):
        getattr(lib, name).argtypes = [vp, i64, vp, vp, vp, vp, vp] + (
            [vp] if name == "ewald_eval_combined_parts" else []) + [vp, i64, vp]
    for name in ("ewald_spread", "ewald_far_grid"):
        getattr(lib, name).argtypes = [vp, i64, vp, vp, vp, i64, vp, i64, vp]
    lib.ewald_count_pairs.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp]
    lib.ewald_stage_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    lib.ewald_debug_fail_next.argtypes = [i32]
    lib.ewald_last_error.restype = ctypes.c_char_p
    lib.ewald_version.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        raise EwaldError(rc, load().ewald_last_error().decode())
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_particles(x, f):
    import torch

    for name, a in (("x", x), ("f", f)):
        if not isinstance(a, torch.Tensor) or a.dtype != torch.float64 or a.dim() != 2 or a.shape[0] != 3:
            raise ValueError("%s must be a (3, n) float64 tensor" % name)
        if not a.is_cuda or not a.is_contiguous():
            raise ValueError("%s must be a contiguous device tensor" % name)
    if x.shape != f.shape:
        raise ValueError("x and f must have the same shape")
    return x.shape[1]


def make_params(box, tol, xi=None, r_c=None, grid=None, P=None, precision="fp64", n_max=1 << 20,
                window_shape=None, p2p_fp64_acc=False, timers=False, window="gaussian", deterministic=False,
                stresslet=False, check_inputs=False):
    """The ewald_params struct for these arguments (None = derive from tol)."""
    p = Params()
    for d in range(3):
        p.box[d] = float(box[d])
        p.grid[d] = int(grid[d]) if grid is not None else 0
    p.xi = float(xi) if xi else 0.0
    p.r_c = float(r_c) if r_c else 0.0
    p.P = int(P) if P else 0
    p.tol = float(tol)
    mode = {"fp64": EWALD_FP64, "fp32": EWALD_FP32_BULK}[precision]
    if window not in ("gaussian", "kb"):
        raise ValueError("window must be 'gaussian' or 'kb'")
    p.precision = mode | (EWALD_FLAG_P2P_FP64_ACC if p2p_fp64_acc else 0) | (
        EWALD_FLAG_STAGE_TIMERS if timers else 0) | (EWALD_FLAG_WINDOW_KB if window == "kb" else 0) | (
        EWALD_FLAG_DETERMINISTIC if deterministic else 0) | (EWALD_FLAG_STRESSLET if stresslet else 0) | (
        EWALD_FLAG_CHECK_INPUTS if check_inputs else 0)
    p.reserved = 0
    p.n_max = int(n_max)
    p.window_shape = float(window_shape) if window_shape else 0.0
    return p


def _info_dict(info, precision):
    q = info.params
    return {
        "box": tuple(q.box), "xi": q.xi, "r_c": q.r_c, "grid": tuple(q.grid), "P": q.P, "tol": q.tol,
        "precision": precision, "mode_flags": q.precision, "n_max": q.n_max, "window_shape": q.window_shape,
        "h": tuple(info.h), "err_near": info.err_near, "err_far": info.err_far,
        "err_window": info.err_window, "tile": info.tile, "n_tiles": tuple(info.n_tiles),
        "stencil": tuple(info.stencil), "workspace_bytes": info.workspace_bytes,
        "fourier_fp64": bool(info.fourier_fp64),
        "predicted_ms": info.predicted_ms,
        "self_coef": info.self_coef,
        "grid_bytes": info.grid_bytes,
        "window": "kb" if q.precision & EWALD_FLAG_WINDOW_KB else "gaussian",
        "deterministic": bool(q.precision & EWALD_FLAG_DETERMINISTIC),
        "stresslet": bool(q.precision & EWALD_FLAG_STRESSLET),
    }


def resolve(box, tol, precision="fp64", **kw):
    """Host-only parameter resolution (no device): the dict a Plan would report."""
    info = PlanInfo()
    p = make_params(box, tol, precision=precision, **kw)
    _check(load().ewald_resolve(ctypes.byref(p), ctypes.byref(info)))
    return _info_dict(info, precision)


class Plan:
    """A resolved spectral Ewald plan (parameters, tables) for one box and tolerance.

    ``precision``: "fp64" or "fp32" (FP32 bulk).  Parameters left as None are derived
    from ``tol`` (Sec. 2.4).  Owns a cached workspace for ``eval`` calls that do not
    pass their own.
    """

    def __init__(self, box, tol, xi=None, r_c=None, grid=None, P=None, precision="fp64", n_max=1 << 20,
                 window_shape=None, p2p_fp64_acc=False, timers=False, window="gaussian", deterministic=False,
                 stresslet=False, check_inputs=False):
        lib = load()
        p = make_params(box, tol, xi, r_c, grid, P, precision, n_max, window_shape, p2p_fp64_acc, timers,
                        window, deterministic, stresslet, check_inputs)
        self._lib = lib  # kept so that the plan can be freed during interpreter shutdown
        h = ctypes.c_void_p()
        _check(lib.ewald_plan_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._ws = None
        info = PlanInfo()
        _check(lib.ewald_plan_get_info(self._h, ctypes.byref(info)))
        self.info = _info_dict(info, precision)
        self.precision = precision

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ewald_plan_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def self_coef(self):
        """c of the self term -c f (the library's value, ewald_plan_info.self_coef)."""
        return self.info["self_coef"]

    def workspace_bytes(self, n):
        return _check(load().ewald_workspace_bytes(self._h, int(n)))

    def workspace(self, n, device=None):
        import torch

        need = self.workspace_bytes(n)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def _ws_args(self, n, workspace, device):
        ws = workspace if workspace is not None else self.workspace(n, device)
        return _ptr(ws), ctypes.c_int64(ws.numel())

    def eval(self, x, f, out=None, workspace=None, stream=None):
        """u (3, n) float64 on the device: the periodic Stokeslet sum at every particle."""
        import torch

        n = _check_particles(x, f)
        u = out if out is not None else torch.empty_like(x)
        wp, wb = self._ws_args(n, workspace, x.device)
        _check(load().ewald_eval(self._h, n, _ptr(x), _ptr(f), _ptr(u), wp, wb, _stream_handle(stream)))
        return u

    @staticmethod
    def _offsets(sizes):
        off = (ctypes.c_int64 * (len(sizes) + 1))()
        for k, m in enumerate(sizes):
            off[k + 1] = off[k] + int(m)
        return off

    def workspace_bytes_batch(self, sizes):
        return _check(load().ewald_workspace_bytes_batch(self._h, len(sizes), self._offsets(sizes)))

    def eval_batch(self, x, f, sizes, out=None, workspace=None, stream=None):
        """u for independent systems sharing this plan: system k is the next sizes[k]
        columns of x and f ((3, sum(sizes)) device arrays), summed over its own images."""
        import torch

        n = _check_particles(x, f)
        if sum(int(m) for m in sizes) != n:
            raise ValueError("sizes must add up to the number of particles")
        u = out if out is not None else torch.empty_like(x)
        off = self._offsets(sizes)
        need = self.workspace_bytes_batch(sizes)
        if workspace is None:
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
            workspace = self._ws
        _check(load().ewald_eval_batch(self._h, len(sizes), off, _ptr(x), _ptr(f), _ptr(u), _ptr(workspace),
                                       ctypes.c_int64(workspace.numel()), _stream_handle(stream)))
        return u

    def eval_noalloc(self, x, f, out=None, stream=None):
        """eval without a caller workspace: the library's built-in scratch array serves
        (at most NOALLOC_MAX_WORKSPACE bytes); calls overlapping on one device race."""
        import torch

        n = _check_particles(x, f)
        u = out if out is not None else torch.empty_like(x)
        _check(load().ewald_eval_noalloc(self._h, n, _ptr(x), _ptr(f), _ptr(u), _stream_handle(stream)))
        return u

    def eval_overlap(self, x, f, out=None, workspace=None, stream=None, near_stream=None):
        """eval with P2P on a second stream beside P2G and the FFTs (joined before G2P).
        The plan keeps one second stream and a pair of events for calls without
        `near_stream`; concurrent calls on other streams pass their own."""
        import torch

        n = _check_particles(x, f)
        u = out if out is not None else torch.empty_like(x)
        wp, wb = self._ws_args(n, workspace, x.device)
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        if near_stream is None:
            if getattr(self, "_near", None) is None:
                self._near = torch.cuda.Stream(device=x.device)  # default priority
            near_stream = self._near
        evs = self._overlap_events(near_stream)
        _check(load().ewald_eval_overlap(self._h, n, _ptr(x), _ptr(f), _ptr(u), wp, wb, _stream_handle(s),
                                         _stream_handle(near_stream), ctypes.c_void_p(evs[0].cuda_event),
                                         ctypes.c_void_p(evs[1].cuda_event)))
        return u

    def _overlap_events(self, near_stream):
        """Fork and join events for overlapped calls using `near_stream` (created once and
        recorded once so that the HIP events exist)."""
        import torch

        cache = self.__dict__.setdefault("_ov_events", {})
        key = near_stream.cuda_stream
        if key not in cache:
            evs = (torch.cuda.Event(), torch.cuda.Event())
            for e in evs:
                e.record(near_stream)
            cache[key] = evs
        return cache[key]

    def eval_parts(self, x, f, workspace=None, stream=None):
        """(u_near, u_far): the P2P sum and the interpolated far field, caller order."""
        import torch

        n = _check_particles(x, f)
        un, uf = torch.empty_like(x), torch.empty_like(x)
        wp, wb = self._ws_args(n, workspace, x.device)
        _check(load().ewald_eval_parts(self._h, n, _ptr(x), _ptr(f), _ptr(un), _ptr(uf), wp, wb,
                                       _stream_handle(stream)))
        return un, uf

    def eval_combined(self, x, f, q, nrm, out=None, workspace=None, stream=None):
        """u (3, n): Stokeslet forces f plus stresslet sources q n^T at every particle
        (plan created with ``stresslet=True``)."""
        import torch

        n = _check_particles(x, f)
        _check_particles(q, nrm)
        if q.shape != x.shape:
            raise ValueError("q and nrm must have the shape of x")
        u = out if out is not None else torch.empty_like(x)
        wp, wb = self._ws_args(n, workspace, x.device)
        _check(load().ewald_eval_combined(self._h, n, _ptr(x), _ptr(f), _ptr(q), _ptr(nrm), _ptr(u), wp, wb,
                                          _stream_handle(stream)))
        return u

    def eval_combined_parts(self, x, f, q, nrm, workspace=None, stream=None):
        """(u_near, u_far) of eval_combined."""
        import torch

        n = _check_particles(x, f)
        _check_particles(q, nrm)
        if q.shape != x.shape:
            raise ValueError("q and nrm must have the shape of x")
        un, uf = torch.empty_like(x), torch.empty_like(x)
        wp, wb = self._ws_args(n, workspace, x.device)
        _check(load().ewald_eval_combined_parts(self._h, n, _ptr(x), _ptr(f), _ptr(q), _ptr(nrm), _ptr(un),
                                                _ptr(uf), wp, wb, _stream_handle(stream)))
        return un, uf

    def _grid_call(self, fn, x, f, workspace, stream):
        import torch

        n = _check_particles(x, f)
        M = self.info["grid"]
        dt = torch.float64 if self.info["fourier_fp64"] else torch.float32
        g = torch.empty((3, M[0], M[1], M[2]), dtype=dt, device=x.device)
        wp, wb = self._ws_args(n, workspace, x.device)
        _check(fn(self._h, n, _ptr(x), _ptr(f), _ptr(g), ctypes.c_int64(g.numel() * g.element_size()), wp, wb,
                  _stream_handle(stream)))
        return g

    def spread(self, x, f, workspace=None, stream=None):
        """The P2G grid phi (3, M1, M2, M3) of eq. (p2g)."""
        return self._grid_call(load().ewald_spread, x, f, workspace, stream)

    def far_grid(self, x, f, workspace=None, stream=None):
        """h1 h2 h3 * v(g_l): the grid G2P interpolates (after FFT, CNV, IFFT)."""
        return self._grid_call(load().ewald_far_grid, x, f, workspace, stream)

    def count_pairs(self, x, f, workspace=None, stream=None):
        """Exact number of ordered pairs within r_c (all images, i != j): the near-field sum's
        pairs.  Synchronises the stream to read the device counter."""
        import torch

        n = _check_particles(x, f)
        c = torch.zeros(1, dtype=torch.int64, device=x.device)
        wp, wb = self._ws_args(n, workspace, x.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(load().ewald_count_pairs(self._h, n, _ptr(x), _ptr(f), _ptr(c), wp, wb, _stream_handle(s)))
        s.synchronize()
        return int(c.item())

    def stage_ms(self):
        """Per-stage device ms of the last evaluation (plan created with timers=True)."""
        buf = (ctypes.c_float * len(STAGES))()
        k = _check(load().ewald_stage_ms(self._h, buf, len(STAGES)))
        return dict(zip(STAGES[:k], [float(v) for v in buf[:k]]))


def debug_fail_next(count=1):
    """Make the next `count` evaluation calls of this thread fail with EWALD_EHIP before
    launching anything (tests of error handling)."""
    _check(load().ewald_debug_fail_next(int(count)))


def version():
    return load().ewald_version().decode()
