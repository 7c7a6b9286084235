"""Thin ctypes binding of libdehaze.so (include/dehaze.h).

Only argument marshalling lives here: torch tensors provide device memory and
the current HIP stream, every computation runs in the library's kernels.  If
the library has not been built, importing this module raises ImportError:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint8, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdehaze.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, ENONFINITE = 0, -1, -2, -3, -4, -5
U8, F32 = 0, 1
HWC, CHW = 0, 1
PAPER_EXPLICIT, JACOBI, PICARD_KRYLOV = 0, 1, 2
U_F32, U_F64 = 0, 1
SCHEMES = {"explicit": PAPER_EXPLICIT, "jacobi": JACOBI, "picard": PICARD_KRYLOV}


class Params(ctypes.Structure):
    _fields_ = [
        ("patch", c_int32), ("g_radius", c_int32),
        ("omega", c_double), ("t0", c_double), ("eps", c_double), ("sigma", c_double),
        ("lambda0", c_double), ("beta_lambda", c_double), ("tau", c_double), ("theta", c_double),
        ("rel_tol", c_double), ("inner_rtol", c_double),
        ("scheme", c_int32), ("max_outer", c_int32), ("max_inner", c_int32), ("check_every", c_int32),
        ("atm_divisor", c_int32), ("warm_start", c_int32), ("nonlocal_term", c_int32),
        ("adaptive", c_int32), ("edge_preserving", c_int32), ("sweeps_per_launch", c_int32),
        ("inner_refine", c_int32), ("strip_rows", c_int32), ("lane_columns", c_int32),
        ("stall_window", c_int32), ("guided_radius", c_int32), ("dark_scales", c_int32),
        ("guided_eps", c_double), ("u_state", c_int32), ("krylov_rows", c_int32),
        ("ngmres_depth", c_int32), ("reserved", c_int32 * 1),
    ]

    def replace(self, **kw) -> "Params":
        p = Params()
        ctypes.pointer(p)[0] = self
        for k, v in kw.items():
            if k == "scheme" and isinstance(v, str):
                v = SCHEMES[v]
            setattr(p, k, v)
        return p


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer", c_int32), ("converged", c_int32), ("inner", c_int64), ("applications", c_int64),
        ("rel_residual", c_double), ("rel_residual0", c_double), ("A", c_float * 3), ("status", c_int32),
        ("restarts", c_int32), ("stalled", c_int32), ("rel_residual_out", c_double),
    ]

    def as_dict(self) -> dict:
        return {"outer": self.outer, "converged": bool(self.converged), "inner": self.inner,
                "applications": self.applications, "rel_residual": self.rel_residual,
                "rel_residual0": self.rel_residual0, "A": list(self.A), "status": self.status,
                "restarts": self.restarts, "stalled": self.stalled, "rel_residual_out": self.rel_residual_out}


class Image(ctypes.Structure):
    _fields_ = [
        ("I", c_void_p), ("H", c_int32), ("W", c_int32), ("pitch", c_int32), ("reserved", c_int32),
        ("u", c_void_p), ("t", c_void_p), ("A", c_void_p), ("u0", c_void_p), ("t_out", c_void_p),
        ("A_out", c_void_p),
    ]


class DehazeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2506_08793_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)
_P = POINTER(Params)
_S = POINTER(Stats)

_SIGS = {
    "dehaze_params_default": (c_int, [_P]),
    "dehaze_params_size": (c_size_t, []),
    "dehaze_stats_size": (c_size_t, []),
    "dehaze_ctx_create": (c_int, [POINTER(c_void_p), c_int]),
    "dehaze_ctx_destroy": (None, [c_void_p]),
    "dehaze_last_error": (ctypes.c_char_p, []),
    "dehaze_strerror": (ctypes.c_char_p, [c_int]),
    "dehaze_prior_workspace_size": (c_size_t, [c_int, c_int, _P]),
    "dehaze_prior": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, _P, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_size_t, c_void_p]),
    "dehaze_solve_workspace_size": (c_size_t, [c_int, c_int, _P]),
    "dehaze_solve": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, _P,
                             c_void_p, c_void_p, c_void_p, c_size_t, _S, c_void_p]),
    "dehaze_batch_workspace_size": (c_size_t, [c_int, POINTER(Image), _P]),
    "dehaze_batch": (c_int, [c_void_p, c_int, POINTER(Image), c_int, c_int, _P, c_void_p, c_size_t, _S, c_void_p]),
    "dehaze_batch_strip_rows": (c_int, [c_void_p, c_int, POINTER(Image), _P, POINTER(c_int), POINTER(c_int)]),
    "dehaze_cnn_param_count": (c_size_t, []),
    "dehaze_cnn_set_weights": (c_int, [c_void_p, c_void_p, c_size_t]),
    "dehaze_cnn_get_weights": (c_int, [c_void_p, c_void_p, c_size_t]),
    "dehaze_cnn_workspace_size": (c_size_t, [c_int, c_int, c_int, c_int]),
    "dehaze_cnn_forward": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]),
    "dehaze_cnn_grad": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "dehaze_cnn_train_step": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                      ctypes.c_float, POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "dehaze_sweep_shape": (c_int, [c_void_p, c_int, c_int, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
    "dehaze_residual_workspace_size": (c_size_t, [c_int, c_int, _P]),
    "dehaze_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, _P, c_void_p,
                                POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "dehaze_residual_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, _P, c_void_p,
                                        c_void_p, c_void_p]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

if _lib.dehaze_params_size() != ctypes.sizeof(Params) or _lib.dehaze_stats_size() != ctypes.sizeof(Stats):
    raise ImportError("dehaze_params / dehaze_stats layout mismatch between binding and library")

EXPORTED = tuple(_SIGS)


def lib():
    return _lib


def _check(rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        raise DehazeError(rc, _lib.dehaze_last_error().decode() or _lib.dehaze_strerror(rc).decode())
    return rc


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def dehaze_params_default(**kw) -> Params:
    p = Params()
    _check(_lib.dehaze_params_default(ctypes.byref(p)))
    return p.replace(**kw) if kw else p


class Context:
    """Owns a dehaze_ctx on one device."""

    def __init__(self, device: int = 0):
        h = c_void_p()
        _check(_lib.dehaze_ctx_create(ctypes.byref(h), device))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _lib.dehaze_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _image_args(I: torch.Tensor, layout: str):
    """(dtype, layout, H, W, pitch) of a device image; strides of size-1 dims are ignored."""
    if not I.is_cuda:
        raise ValueError("image must be a device tensor")
    dtype = {torch.uint8: U8, torch.float32: F32}[I.dtype]
    if layout == "CHW":
        _, H, W = I.shape
        pitch = I.stride(1) if H > 1 else W
        if (W > 1 and I.stride(2) != 1) or I.stride(0) != H * pitch or pitch < W:
            raise ValueError("CHW image must be row-contiguous with planes packed")
        return dtype, CHW, H, W, pitch
    H, W, _ = I.shape
    pitch = I.stride(0) // 3 if H > 1 else W
    if I.stride(2) != 1 or (W > 1 and I.stride(1) != 3) or (H > 1 and I.stride(0) % 3) or pitch < W:
        raise ValueError("HWC image must be pixel-contiguous")
    return dtype, HWC, H, W, pitch


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def dehaze_prior(ctx: Context, I: torch.Tensor, params: Params = None, A_in: torch.Tensor = None,
                 layout: str = "CHW", outputs=("dark", "t_d", "t", "lam", "phi")) -> dict:
    """Front end: returns the requested outputs plus A (3 floats) as device tensors."""
    p = params or dehaze_params_default()
    dtype, lay, H, W, pitch = _image_args(I, layout)
    dev = I.device
    out = {}
    for name in outputs:
        shape = (3, H, W) if name == "phi" else (H, W)
        out[name] = torch.empty(shape, dtype=torch.uint8 if name == "dark_u8" else torch.float32, device=dev)
    A = torch.empty(3, dtype=torch.float32, device=dev)
    ws = _workspace(_lib.dehaze_prior_workspace_size(H, W, ctypes.byref(p)), dev)
    _check(_lib.dehaze_prior(ctx.handle, I.data_ptr(), dtype, lay, H, W, pitch, ctypes.byref(p), _ptr(A_in),
                             _ptr(out.get("dark")), _ptr(out.get("dark_u8")), _ptr(out.get("t_d")),
                             _ptr(out.get("t")), _ptr(out.get("lam")), _ptr(out.get("phi")), A.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream()))
    out["A"] = A
    out["_ws"] = ws  # keeps the workspace alive until the caller synchronises
    return out


def dehaze_solve(ctx: Context, I: torch.Tensor, t: torch.Tensor, A: torch.Tensor, params: Params = None,
                 u0: torch.Tensor = None, u: torch.Tensor = None, layout: str = "CHW", stats: bool = True,
                 ws: torch.Tensor = None):
    """Solve the PDE for one image; returns (u, stats dict or None)."""
    p = params or dehaze_params_default()
    dtype, lay, H, W, pitch = _image_args(I, layout)
    dev = I.device
    for name, tens, shape in (("t", t, (H, W)), ("A", A, (3,)), ("u0", u0, (3, H, W))):
        if tens is not None and (tuple(tens.shape) != shape or not tens.is_contiguous()
                                 or tens.dtype != torch.float32 or not tens.is_cuda):
            raise ValueError(f"{name} must be a contiguous float32 device tensor of shape {shape}")
    u_dtype = torch.float64 if p.u_state == U_F64 else torch.float32
    if u is None:
        u = torch.empty((3, H, W), dtype=u_dtype, device=dev)
    elif u.dtype != u_dtype or tuple(u.shape) != (3, H, W) or not u.is_contiguous():
        raise ValueError(f"u must be a contiguous {u_dtype} tensor of shape {(3, H, W)}")
    need = _lib.dehaze_solve_workspace_size(H, W, ctypes.byref(p))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    st = Stats() if stats else None
    rc = _lib.dehaze_solve(ctx.handle, I.data_ptr(), dtype, lay, H, W, pitch, t.data_ptr(), A.data_ptr(),
                           ctypes.byref(p), _ptr(u0), u.data_ptr(), ws.data_ptr(), ws.numel(),
                           ctypes.byref(st) if st is not None else None, _stream())
    _check(rc, allow=(OK, ENOTCONV))
    return u, (st.as_dict() if st is not None else None)


def solve_workspace(H: int, W: int, params: Params, device="cuda") -> torch.Tensor:
    return _workspace(_lib.dehaze_solve_workspace_size(H, W, ctypes.byref(params)), device)


def dehaze_residual(ctx: Context, u: torch.Tensor, phi: torch.Tensor, lam: torch.Tensor, params: Params = None,
                    want_r: bool = False):
    """rho = ||Phi - L_{D(u)} u|| / ||Phi||; returns (rho, r or None)."""
    p = params or dehaze_params_default()
    _, H, W = u.shape
    for tens in (u, phi, lam):
        if not (tens.is_cuda and tens.is_contiguous() and tens.dtype == torch.float32):
            raise ValueError("u, phi, lam must be contiguous float32 device tensors")
    r = torch.empty_like(u) if want_r else None
    ws = _workspace(_lib.dehaze_residual_workspace_size(H, W, ctypes.byref(p)), u.device)
    rho = c_double()
    _check(_lib.dehaze_residual(ctx.handle, u.data_ptr(), phi.data_ptr(), lam.data_ptr(), H, W, ctypes.byref(p),
                                _ptr(r), ctypes.byref(rho), ws.data_ptr(), ws.numel(), _stream()))
    return rho.value, r


def dehaze_residual_noalloc(ctx: Context, u: torch.Tensor, phi: torch.Tensor, lam: torch.Tensor,
                            rho: torch.Tensor, params: Params = None, r: torch.Tensor = None) -> None:
    """Allocation-free rho into the one-element float64 device tensor `rho`
    (and Phi - L u into `r` when given); enqueued on the current stream, no
    synchronisation.  The caller provides every output."""
    p = params or dehaze_params_default()
    _, H, W = u.shape
    for tens in (u, phi, lam) + (() if r is None else (r,)):
        if not (tens.is_cuda and tens.is_contiguous() and tens.dtype == torch.float32):
            raise ValueError("u, phi, lam and r must be contiguous float32 device tensors")
    if not (rho.is_cuda and rho.dtype == torch.float64 and rho.numel() >= 1):
        raise ValueError("rho must be a float64 device tensor")
    _check(_lib.dehaze_residual_noalloc(ctx.handle, u.data_ptr(), phi.data_ptr(), lam.data_ptr(), H, W,
                                        ctypes.byref(p), _ptr(r), rho.data_ptr(), _stream()))


def dehaze_batch(ctx: Context, images, params: Params = None, layout: str = "CHW", t=None, A=None, u0=None,
                 want_t: bool = False, stats: bool = True, ws: torch.Tensor = None, outs=None,
                 allow_nonfinite: bool = False):
    """Solve a list of device images (each CHW (3,H,W) or HWC (H,W,3), one dtype).

    t, A, u0: optional per-image lists (None entries are estimated / Phi).
    allow_nonfinite: return normally when an image met a non-finite value (its
    stats entry says which) instead of raising.
    Returns (list of u, list of stats dicts or None, list of t or None, list of A).
    """
    p = params or dehaze_params_default()
    n = len(images)
    arr = (Image * n)()
    keep = []
    us, ts, As = [], [], []
    dtype0 = None
    for i, I in enumerate(images):
        dtype, lay, H, W, pitch = _image_args(I, layout)
        if dtype0 is None:
            dtype0, lay0 = dtype, lay
        elif dtype != dtype0:
            raise ValueError("all images of a batch share one dtype")
        u_dtype = torch.float64 if p.u_state == U_F64 else torch.float32
        u = outs[i] if outs is not None else torch.empty((3, H, W), dtype=u_dtype, device=I.device)
        if u.dtype != u_dtype or tuple(u.shape) != (3, H, W) or not u.is_contiguous():
            raise ValueError(f"output {i} must be a contiguous {u_dtype} tensor of shape {(3, H, W)}")
        ti = None if t is None else t[i]
        Ai = None if A is None else A[i]
        ui = None if u0 is None else u0[i]
        t_out = torch.empty((H, W), dtype=torch.float32, device=I.device) if (want_t and ti is None) else None
        A_out = torch.empty(3, dtype=torch.float32, device=I.device) if Ai is None else None
        arr[i] = Image(I.data_ptr(), H, W, pitch, 0, u.data_ptr(), _ptr(ti), _ptr(Ai), _ptr(ui), _ptr(t_out),
                       _ptr(A_out))
        keep += [ti, Ai, ui]
        us.append(u)
        ts.append(t_out if ti is None else ti)
        As.append(A_out if Ai is None else Ai)
    need = _lib.dehaze_batch_workspace_size(n, arr, ctypes.byref(p))
    if need == 0:
        raise DehazeError(EINVAL, "bad batch description")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, images[0].device)
    st = (Stats * n)() if stats else None
    rc = _lib.dehaze_batch(ctx.handle, n, arr, dtype0, lay0, ctypes.byref(p), ws.data_ptr(), ws.numel(),
                           st if st is not None else None, _stream())
    _check(rc, allow=(OK, ENOTCONV, ENONFINITE) if allow_nonfinite else (OK, ENOTCONV))
    return us, ([x.as_dict() for x in st] if st is not None else None), ts, As


def batch_workspace_bytes(shapes, params: Params = None) -> int:
    p = params or dehaze_params_default()
    n = len(shapes)
    arr = (Image * n)()
    for i, (H, W) in enumerate(shapes):
        arr[i] = Image(1, H, W, W, 0, 1, None, None, None, None, None)
    return int(_lib.dehaze_batch_workspace_size(n, arr, ctypes.byref(p)))


def dehaze_batch_strip_rows(ctx, shapes, params: Params = None):
    """(rows per image, tuned) of the BiCGSTAB strip kernels for a batch of
    (H, W) shapes; ctx may be None (the size rule alone)."""
    p = params or dehaze_params_default()
    n = len(shapes)
    arr = (Image * n)()
    for i, (H, W) in enumerate(shapes):
        arr[i] = Image(1, H, W, W, 0, 1, None, None, None, None, None)
    rows = (c_int * n)()
    tuned = c_int()
    _check(_lib.dehaze_batch_strip_rows(None if ctx is None else ctx.handle, n, arr, ctypes.byref(p), rows,
                                        ctypes.byref(tuned)))
    return list(rows), bool(tuned.value)


# ---------------------------------------------------------------- network
def dehaze_cnn_param_count() -> int:
    return int(_lib.dehaze_cnn_param_count())


def dehaze_cnn_set_weights(ctx: Context, w) -> None:
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(_lib.dehaze_cnn_set_weights(ctx.handle, w.ctypes.data, w.size))


def dehaze_cnn_get_weights(ctx: Context):
    import numpy as np
    w = np.empty(dehaze_cnn_param_count(), dtype=np.float32)
    _check(_lib.dehaze_cnn_get_weights(ctx.handle, w.ctypes.data, w.size))
    return w


def _cnn_args(I, t, A):
    n, c, H, W = I.shape
    for x, shape in ((I, (n, 3, H, W)), (t, (n, H, W)), (A, (n, 3))):
        if tuple(x.shape) != shape or not x.is_contiguous() or x.dtype != torch.float32 or not x.is_cuda:
            raise ValueError(f"expected a contiguous float32 device tensor of shape {shape}")
    return n, H, W


def cnn_workspace(n, H, W, training: bool, device="cuda") -> torch.Tensor:
    return _workspace(_lib.dehaze_cnn_workspace_size(n, H, W, 1 if training else 0), device)


def dehaze_cnn_forward(ctx: Context, I, t, A, ws=None):
    n, H, W = _cnn_args(I, t, A)
    u = torch.empty((n, 3, H, W), dtype=torch.float32, device=I.device)
    need = _lib.dehaze_cnn_workspace_size(n, H, W, 0)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, I.device)
    _check(_lib.dehaze_cnn_forward(ctx.handle, n, H, W, I.data_ptr(), t.data_ptr(), A.data_ptr(), u.data_ptr(),
                                   ws.data_ptr(), ws.numel(), _stream()))
    return u


def dehaze_cnn_grad(ctx: Context, I, t, A, target, ws=None):
    n, H, W = _cnn_args(I, t, A)
    g = torch.empty(dehaze_cnn_param_count(), dtype=torch.float32, device=I.device)
    need = _lib.dehaze_cnn_workspace_size(n, H, W, 1)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, I.device)
    loss = c_double()
    _check(_lib.dehaze_cnn_grad(ctx.handle, n, H, W, I.data_ptr(), t.data_ptr(), A.data_ptr(), target.data_ptr(),
                                g.data_ptr(), ctypes.byref(loss), ws.data_ptr(), ws.numel(), _stream()))
    return g, loss.value


def dehaze_cnn_train_step(ctx: Context, I, t, A, target, lr: float, ws=None, want_loss: bool = True):
    n, H, W = _cnn_args(I, t, A)
    need = _lib.dehaze_cnn_workspace_size(n, H, W, 1)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, I.device)
    loss = c_double()
    _check(_lib.dehaze_cnn_train_step(ctx.handle, n, H, W, I.data_ptr(), t.data_ptr(), A.data_ptr(),
                                      target.data_ptr(), float(lr), ctypes.byref(loss) if want_loss else None,
                                      ws.data_ptr(), ws.numel(), _stream()))
    return loss.value if want_loss else None


def dehaze_sweep_shape(ctx: Context, H: int, W: int, scheme: int = JACOBI):
    """(sweeps per launch, strip rows, columns per lane) the context's tuner
    chose for H x W sweeps ((0, 0, 0) if none yet)."""
    k, srows, cols = c_int(), c_int(), c_int()
    _check(_lib.dehaze_sweep_shape(ctx.handle, H, W, scheme, ctypes.byref(k), ctypes.byref(srows), ctypes.byref(cols)))
    return k.value, srows.value, cols.value
