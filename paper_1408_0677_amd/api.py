"""Python binding of the C ABI in include/mls.h (argument marshalling only).

Device memory and streams come from PyTorch: inputs and outputs are CUDA
(HIP) tensors, the stream is torch's current stream unless one is passed.
Every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import threading

from . import _lib

BASIS = {"constant": 0, "linear": 1, "quadratic": 2, "rigid": 3}
WEIGHT = {"gaussian": 0, "wendland": 1, "invpow": 2}
PRECISION = {"f64": 0, "bf16": 1, "fp16": 2}
STATUS_OK = 0
DEGREE_UNDETERMINED = 255


class MlsError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib.load()
        name = lib.mls_status_string(status).decode()
        detail = lib.mls_last_error().decode()
        super().__init__(f"{where}: {name}: {detail}")
        self.status = status
        self.name = name


def _check(status: int, where: str):
    if status != STATUS_OK:
        raise MlsError(status, where)


class Context:
    """An mls_context on one device (default: torch's current device)."""

    def __init__(self, device: int | None = None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._ptr = ctypes.c_void_p()
        _check(_lib.load().mls_context_create(self.device, ctypes.byref(self._ptr)),
               "mls_context_create")

    @property
    def handle(self):
        return self._ptr

    def trace(self, enable: bool = True, jsonl_path: str | None = None):
        """Per-stage timing of this context's calls (mls_context_trace); with
        ``jsonl_path`` one JSON line per call is appended there."""
        _check(_lib.load().mls_context_trace(self._ptr, 1 if enable else 0,
                                             None if jsonl_path is None
                                             else str(jsonl_path).encode()),
               "mls_context_trace")

    def trace_last(self) -> dict:
        """Stage times (ms) of the last traced call: {"call", "stages": {name:
        ms}, "total_ms"}; waits for the traced calls to finish."""
        rec = _lib.MlsTraceRecord()
        _check(_lib.load().mls_context_trace_last(self._ptr, ctypes.byref(rec)),
               "mls_context_trace_last")
        stages = {bytes(rec.stage[k].value).decode(): float(rec.ms[k])
                  for k in range(rec.n_stages)}
        return {"call": rec.call.decode(), "form": int(rec.form), "stages": stages,
                "total_ms": float(rec.total_ms)}

    def close(self):
        if self._ptr:
            _lib.load().mls_context_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = threading.local()


def default_context(device: int | None = None) -> Context:
    """The calling thread's context on ``device``.  A context serves one host
    thread at a time, so each thread gets its own; calls on one context that
    use different streams are ordered by the library itself."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    per_thread = getattr(_default_ctx, "by_device", None)
    if per_thread is None:
        per_thread = _default_ctx.by_device = {}
    if dev not in per_thread:
        per_thread[dev] = Context(dev)
    return per_thread[dev]


def _require(t, name: str, dtype, device=None, numel: int | None = None, shape=None):
    """Refuse anything but a contiguous device tensor of ``dtype`` (and, when
    given, on ``device``, with ``numel`` elements or exactly ``shape``): a
    wrong buffer would make a kernel read or write past its end."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, not {t.numel()}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")


def _points_values(points, values):
    """Checked (points (N, 2), values (N, D)) float32 device tensors."""
    import torch
    _require(points, "points", torch.float32)
    if points.dim() != 2 or points.shape[1] != 2:
        raise ValueError(f"points must have shape (N, 2), not {tuple(points.shape)}")
    _require(values, "values", torch.float32, device=points.device)
    if values.dim() == 1:
        values = values.view(-1, 1)
    if values.dim() != 2:
        raise ValueError(f"values must have shape (N, D), not {tuple(values.shape)}")
    if values.shape[0] != points.shape[0]:
        raise ValueError(f"points hold {points.shape[0]} rows, values {values.shape[0]}")
    return points, values


def grid_struct(grid: dict) -> _lib.MlsGrid:
    return _lib.MlsGrid(float(grid["x0"]), float(grid["y0"]), float(grid["dx"]),
                        float(grid["dy"]), int(grid["width"]), int(grid["height"]))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def fit(points, values, grid: dict, basis: str = "linear", weight: str = "gaussian",
        h: float = 0.05, alpha: float = 1.0, precision: str = "f64",
        pivot_tol: float = 1e-8, weight_floor: float = 1e-6, lp_terms: int = 0, out=None,
        degree_out=None, want_degree: bool = True, ctx: Context | None = None,
        stream=None, lp_slab: int = 0, lp_form: int = 0):
    """MLS fields of ``values`` (N, D) at the nodes of ``grid``.

    ``points`` float32 (N, 2) and ``values`` float32 (N, D) are contiguous
    device tensors.  Returns ``(fields (D, H, W) float32, degree (H, W)
    uint8 or None)``; ``out`` / ``degree_out`` may supply the buffers.
    """
    import torch
    points, values = _points_values(points, values)
    n, d = values.shape
    W, H = int(grid["width"]), int(grid["height"])
    if out is None:
        out = torch.empty((d, H, W), dtype=torch.float32, device=points.device)
    else:
        _require(out, "out", torch.float32, device=points.device, numel=d * H * W)
    if degree_out is None and want_degree:
        degree_out = torch.empty((H, W), dtype=torch.uint8, device=points.device)
    elif degree_out is not None:
        _require(degree_out, "degree_out", torch.uint8, device=points.device, numel=H * W)
    ctx = ctx or default_context(points.device.index)
    g = grid_struct(grid)
    wt = _lib.MlsWeight(WEIGHT[weight], float(h), float(alpha))
    opts = _lib.MlsSolveOpts(float(pivot_tol), float(weight_floor), int(lp_terms),
                             int(lp_slab), int(lp_form))
    st = _lib.load().mls_fit(ctx.handle, _ptr(points), _ptr(values), n, d, BASIS[basis],
                             ctypes.byref(wt), ctypes.byref(g), PRECISION[precision],
                             ctypes.byref(opts), _ptr(out), _ptr(degree_out),
                             _stream_handle(stream))
    _check(st, "mls_fit")
    return out, degree_out


def fit_grad(points, values, grid: dict, basis: str = "linear", weight: str = "gaussian",
             h: float = 0.05, alpha: float = 1.0, precision: str = "f64",
             pivot_tol: float = 1e-8, weight_floor: float = 1e-6, lp_terms: int = 0,
             lp_slab: int = 0, ctx: Context | None = None, stream=None):
    """As ``fit``, plus the slopes of the local fits: returns ``(fields (D, H,
    W), grads (D, 2, H, W), degree (H, W))``; grads[d, 0] = d f_d / dx,
    grads[d, 1] = d f_d / dy."""
    import torch
    points, values = _points_values(points, values)
    n, d = values.shape
    W, H = int(grid["width"]), int(grid["height"])
    out = torch.empty((d, H, W), dtype=torch.float32, device=points.device)
    grads = torch.empty((d, 2, H, W), dtype=torch.float32, device=points.device)
    degree = torch.empty((H, W), dtype=torch.uint8, device=points.device)
    ctx = ctx or default_context(points.device.index)
    g = grid_struct(grid)
    wt = _lib.MlsWeight(WEIGHT[weight], float(h), float(alpha))
    opts = _lib.MlsSolveOpts(float(pivot_tol), float(weight_floor), int(lp_terms),
                             int(lp_slab))
    st = _lib.load().mls_fit_grad(ctx.handle, _ptr(points), _ptr(values), n, d, BASIS[basis],
                                  ctypes.byref(wt), ctypes.byref(g), PRECISION[precision],
                                  ctypes.byref(opts), _ptr(out), _ptr(grads), _ptr(degree),
                                  _stream_handle(stream))
    _check(st, "mls_fit_grad")
    return out, grads, degree


def layout(pos, mesh: dict, C: float, D: float, eta: float, t0: float, lam: float,
           iterations: int, ctx: Context | None = None, stream=None):
    """Planarity-preserving layout (mls_layout).  ``pos`` float32 (n, 2)
    device tensor, updated in place and returned; ``mesh`` holds int32 device
    tensors adj_start (n+1), adj, fan_start (n+1), fan (T, 2) or flat."""
    import torch
    if not (isinstance(pos, torch.Tensor) and pos.is_cuda and pos.dtype == torch.float32
            and pos.is_contiguous() and pos.dim() == 2 and pos.shape[1] == 2):
        raise ValueError("pos must be a contiguous float32 (n, 2) device tensor")
    n = pos.shape[0]
    for key in ("adj_start", "adj", "fan_start", "fan"):
        t = mesh[key]
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32
                and t.is_contiguous() and t.device == pos.device):
            raise ValueError(f"mesh['{key}'] must be a contiguous int32 tensor on {pos.device}")
    for key in ("adj_start", "fan_start"):
        if mesh[key].numel() != n + 1:
            raise ValueError(f"mesh['{key}'] must hold n + 1 = {n + 1} entries")
    adj, fan = mesh["adj"], mesh["fan"]
    n_adj = int(adj.numel())
    n_fan = int(fan.numel()) // 2
    ctx = ctx or default_context(pos.device.index)
    prm = _lib.MlsLayoutParams(float(C), float(D), float(eta), float(t0), float(lam))
    st = _lib.load().mls_layout(ctx.handle, _ptr(pos), n, _ptr(mesh["adj_start"]),
                                _ptr(adj) if n_adj else None, n_adj, _ptr(mesh["fan_start"]),
                                _ptr(fan) if n_fan else None, n_fan, ctypes.byref(prm),
                                int(iterations), _stream_handle(stream))
    _check(st, "mls_layout")
    return pos


CAPACITY_ERROR = -3


def contour(fields, grid: dict, iso, want_cases: bool = True, want_ids: bool = True,
            capacity: int | None = None, ctx: Context | None = None, stream=None):
    """Marching-squares segments of ``fields`` (D, H, W) at isovalues ``iso``
    (D, n_iso), both float32 device tensors.

    Returns ``(segments (S, 4), ids (S, 3) or None, cases (D, n_iso, H-1,
    W-1) or None)``.  Without ``capacity`` the call first asks for the count
    and then runs again with an exact buffer.
    """
    import torch
    _require(fields, "fields", torch.float32)
    if fields.dim() == 2:
        fields = fields.unsqueeze(0)
    if fields.dim() != 3:
        raise ValueError(f"fields must have shape (D, H, W), not {tuple(fields.shape)}")
    D, H, W = fields.shape
    if (W, H) != (int(grid["width"]), int(grid["height"])):
        raise ValueError(f"fields are {H} x {W}, the grid {grid['height']} x {grid['width']}")
    iso = iso.to(device=fields.device, dtype=torch.float32).reshape(D, -1).contiguous()
    n_iso = iso.shape[1]
    dev = fields.device
    ctx = ctx or default_context(dev.index)
    g = grid_struct(grid)
    cases = (torch.empty((D, n_iso, H - 1, W - 1), dtype=torch.uint8, device=dev)
             if want_cases else None)
    lib = _lib.load()
    count = ctypes.c_int64(0)
    cap = 0 if capacity is None else int(capacity)
    while True:
        segs = torch.empty((max(cap, 1), 4), dtype=torch.float32, device=dev)
        ids = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=dev) if want_ids else None
        st = lib.mls_contour(ctx.handle, _ptr(fields), D, ctypes.byref(g), _ptr(iso), n_iso,
                             _ptr(cases), _ptr(segs) if cap > 0 else None,
                             _ptr(ids) if cap > 0 else None, cap, ctypes.byref(count),
                             _stream_handle(stream))
        if st == CAPACITY_ERROR and (capacity is None or cap == 0):
            cap = int(count.value)
            continue
        _check(st, "mls_contour")
        break
    n = int(count.value)
    return segs[:n], (ids[:n] if ids is not None else None), cases


def map_bands(fields, grid: dict, iso, colormap=None, want_bands: bool = True,
              ctx: Context | None = None, stream=None):
    """Discrete-colour bands (Sec. 3.4, Fig. 5b) of ``fields`` (D, H, W) at
    isovalues ``iso`` (D, n_iso), both float32 device tensors: returns
    ``(bands uint8 (D, H, W) or None, rgba (D, H, W) or None)``; ``colormap``
    (D, n_iso + 1) int32 device tensor of RGBA8 words, one per band."""
    import torch
    _require(fields, "fields", torch.float32)
    if fields.dim() == 2:
        fields = fields.unsqueeze(0)
    D, H, W = fields.shape
    if (W, H) != (int(grid["width"]), int(grid["height"])):
        raise ValueError(f"fields are {H} x {W}, the grid {grid['height']} x {grid['width']}")
    dev = fields.device
    _require(iso, "iso", torch.float32, device=dev)
    if iso.numel() % D or iso.numel() == 0:
        raise ValueError("iso must hold n_iso values per field")
    n_iso = iso.numel() // D
    if colormap is not None:
        # RGBA8 colours packed into 32-bit words (held as int32 tensors)
        _require(colormap, "colormap", torch.int32, device=dev, numel=D * (n_iso + 1))
    bands = torch.empty((D, H, W), dtype=torch.uint8, device=dev) if want_bands else None
    rgba = (torch.empty((D, H, W), dtype=colormap.dtype, device=dev)
            if colormap is not None else None)
    ctx = ctx or default_context(dev.index)
    st = _lib.load().mls_map_bands(ctx.handle, _ptr(fields), D, ctypes.byref(grid_struct(grid)),
                                   _ptr(iso), n_iso, _ptr(colormap), _ptr(bands), _ptr(rgba),
                                   _stream_handle(stream))
    _check(st, "mls_map_bands")
    return bands, rgba


def map_adaptive(fields, grads, grid: dict, levels, n_levels: int = 3, halfwidth: float = 1.0,
                 fade_lo: float = 4.0, fade_hi: float = 12.0, ctx: Context | None = None,
                 stream=None):
    """Adaptive contour-line intensity (Sec. 3.4, Fig. 5d) of ``fields``
    (D, H, W) with their gradients ``grads`` (D, 2, H, W) (as fit_grad
    returns them) and ``levels`` (D, 2) = (origin, spacing) of the level-0
    lines, float32 device tensors.  Returns float32 (D, H, W)."""
    import torch
    _require(fields, "fields", torch.float32)
    if fields.dim() == 2:
        fields = fields.unsqueeze(0)
    D, H, W = fields.shape
    if (W, H) != (int(grid["width"]), int(grid["height"])):
        raise ValueError(f"fields are {H} x {W}, the grid {grid['height']} x {grid['width']}")
    dev = fields.device
    _require(grads, "grads", torch.float32, device=dev, numel=2 * D * H * W)
    _require(levels, "levels", torch.float32, device=dev, numel=2 * D)
    out = torch.empty((D, H, W), dtype=torch.float32, device=dev)
    prm = _lib.MlsAdaptiveParams(int(n_levels), float(halfwidth), float(fade_lo), float(fade_hi))
    ctx = ctx or default_context(dev.index)
    st = _lib.load().mls_map_adaptive(ctx.handle, _ptr(fields), _ptr(grads), D,
                                      ctypes.byref(grid_struct(grid)), _ptr(levels),
                                      ctypes.byref(prm), _ptr(out), _stream_handle(stream))
    _check(st, "mls_map_adaptive")
    return out


def contour_static(fields, grid: dict, iso, segments, count, ids=None, cases=None,
                   ctx: Context | None = None, stream=None):
    """Allocation-free marching squares (mls_contour_static) into caller
    buffers: ``segments`` float32 (capacity, 4), ``count`` int64 (1,) device
    tensor receiving the required segment count, optional ``ids`` int32
    (capacity, 3) and ``cases`` uint8 (D, n_iso, H-1, W-1).  Returns at once;
    the first min(count, capacity) segments are valid once the stream has
    run."""
    import torch
    _require(fields, "fields", torch.float32)
    if fields.dim() == 2:
        fields = fields.unsqueeze(0)
    if fields.dim() != 3:
        raise ValueError(f"fields must have shape (D, H, W), not {tuple(fields.shape)}")
    D, H, W = fields.shape
    if (W, H) != (int(grid["width"]), int(grid["height"])):
        raise ValueError(f"fields are {H} x {W}, the grid {grid['height']} x {grid['width']}")
    dev = fields.device
    _require(iso, "iso", torch.float32, device=dev)
    if iso.numel() % D or iso.numel() == 0:
        raise ValueError("iso must hold n_iso values per field")
    n_iso = iso.numel() // D
    _require(segments, "segments", torch.float32, device=dev)
    if segments.dim() != 2 or segments.shape[1] != 4:
        raise ValueError("segments must have shape (capacity, 4)")
    cap = int(segments.shape[0])
    _require(count, "count", torch.int64, device=dev, numel=1)
    if ids is not None:
        _require(ids, "ids", torch.int32, device=dev, numel=3 * cap)
    if cases is not None:
        _require(cases, "cases", torch.uint8, device=dev, numel=D * n_iso * (H - 1) * (W - 1))
    ctx = ctx or default_context(dev.index)
    g = grid_struct(grid)
    st = _lib.load().mls_contour_static(ctx.handle, _ptr(fields), D, ctypes.byref(g), _ptr(iso),
                                        n_iso, _ptr(cases), _ptr(segments) if cap else None,
                                        _ptr(ids) if cap else None, cap, _ptr(count),
                                        _stream_handle(stream))
    _check(st, "mls_contour_static")
    return segments, count


PENDING = 1


def fit_scratch_bytes(n: int, d: int, grid: dict, precision: str = "f64",
                      weight: str = "gaussian", h: float = 0.05, alpha: float = 1.0) -> int:
    """Device scratch bytes mls_fit needs for such a request."""
    wt = _lib.MlsWeight(WEIGHT[weight], float(h), float(alpha))
    return int(_lib.load().mls_fit_scratch_bytes(int(n), int(d), PRECISION[precision],
                                                 ctypes.byref(wt),
                                                 ctypes.byref(grid_struct(grid))))


class ServerError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib.load()
        name = lib.mls_status_string(status).decode()
        super().__init__(f"{where}: {name}: {lib.mls_server_last_error().decode()}")
        self.status = status
        self.name = name


class Server:
    """The served form (mls_server_*): resident point sets; requests admitted
    as they arrive onto slots, 16-bit Gaussian requests of one kernel class
    batched into persistent kernels.  Output tensors of submitted requests
    must stay alive until their result is collected."""

    def __init__(self, device: int = 0, hbm_budget: int = 2 << 30, slots: int = 4,
                 slot_scratch: int = 64 << 20, tune: bool = False,
                 tuner_cache: str | None = None):
        self._ptr = ctypes.c_void_p()
        st = _lib.load().mls_server_create(int(device), int(hbm_budget), int(slots),
                                           int(slot_scratch), ctypes.byref(self._ptr))
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_create")
        self._keep = {}
        self._sets = {}
        if tune or tuner_cache:
            self.tuning(tune, tuner_cache)

    def tuning(self, enable: bool, cache_path: str | None = None):
        st = _lib.load().mls_server_tuning(self._ptr, 1 if enable else 0,
                                           None if cache_path is None else
                                           str(cache_path).encode())
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_tuning")

    def tuned_classes(self) -> int:
        return int(_lib.load().mls_server_tuned_classes(self._ptr))

    def tuning_pending(self) -> int:
        return int(_lib.load().mls_server_tuning_pending(self._ptr))

    def cancel(self, ticket: int):
        st = _lib.load().mls_server_cancel(self._ptr, int(ticket))
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_cancel")

    def close(self):
        if self._ptr:
            _lib.load().mls_server_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def put_points(self, points, values) -> int:
        import torch
        points, values = _points_values(points, values)
        # the copy reads the tensors now, from the server's own stream: the
        # work that produced them (on torch's stream) must be finished
        torch.cuda.current_stream(points.device).synchronize()
        pid = ctypes.c_uint64()
        st = _lib.load().mls_server_put_points(self._ptr, _ptr(points), _ptr(values),
                                               values.shape[0], values.shape[1],
                                               ctypes.byref(pid))
        if st == STATUS_OK:
            self._sets[int(pid.value)] = (points.device, int(values.shape[1]))
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_put_points")
        return int(pid.value)

    def release_points(self, pointset: int):
        st = _lib.load().mls_server_release_points(self._ptr, int(pointset))
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_release_points")
        self._sets.pop(int(pointset), None)

    def submit(self, pointset: int, grid: dict, out, degree_out=None, basis: str = "linear",
               weight: str = "gaussian", h: float = 0.05, alpha: float = 1.0,
               precision: str = "f64", pivot_tol: float = 1e-8, weight_floor: float = 1e-6,
               lp_terms: int = 0, lp_slab: int = 0, lp_form: int = 0,
               timeout_s: float = 0.0) -> int:
        import torch
        # point sets of this server: the outputs must fit them (an unknown
        # id is left to the library, which refuses it without a launch)
        if int(pointset) in self._sets:
            dev, d = self._sets[int(pointset)]
            W, H = int(grid["width"]), int(grid["height"])
            _require(out, "out", torch.float32, device=dev, numel=d * H * W)
            if degree_out is not None:
                _require(degree_out, "degree_out", torch.uint8, device=dev, numel=H * W)
        # the server writes the outputs from its own streams, which are not
        # ordered with torch's: whatever is still queued on them must finish
        torch.cuda.current_stream(out.device).synchronize()
        req = _lib.MlsRequest(int(pointset), BASIS[basis],
                              _lib.MlsWeight(WEIGHT[weight], float(h), float(alpha)),
                              grid_struct(grid), PRECISION[precision],
                              _lib.MlsSolveOpts(float(pivot_tol), float(weight_floor),
                                                int(lp_terms), int(lp_slab), int(lp_form)),
                              out.data_ptr(),
                              None if degree_out is None else degree_out.data_ptr(),
                              float(timeout_s))
        t = ctypes.c_uint64()
        st = _lib.load().mls_server_submit(self._ptr, ctypes.byref(req), ctypes.byref(t))
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_submit")
        self._keep[int(t.value)] = (out, degree_out)
        return int(t.value)

    @staticmethod
    def _result(res):
        return {"status": int(res.status), "t_submit": res.t_submit, "t_admit": res.t_admit,
                "t_start": res.t_start, "t_end": res.t_end, "detail": res.detail.decode()}

    def poll(self, ticket: int):
        """None while pending, else the result dict."""
        res = _lib.MlsResult()
        st = _lib.load().mls_server_poll(self._ptr, int(ticket), ctypes.byref(res))
        if st == PENDING:
            return None
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_poll")
        self._keep.pop(int(ticket), None)
        return self._result(res)

    def wait(self, ticket: int):
        res = _lib.MlsResult()
        st = _lib.load().mls_server_wait(self._ptr, int(ticket), ctypes.byref(res))
        if st != STATUS_OK:
            raise ServerError(st, "mls_server_wait")
        self._keep.pop(int(ticket), None)
        return self._result(res)
