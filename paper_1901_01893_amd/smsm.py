"""Python binding of libsmsm.so (the C ABI declared in include/smsm.h).

Argument marshalling only: every function hands device pointers of torch
tensors and the current HIP stream to the library; all arithmetic runs in the
library's HIP kernels.  There is no fallback: if the library is not built the
first call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmsm.so")

SMSM_OK = 0
SMSM_E_INVALID = -1
SMSM_E_UNSUPPORTED = -2
SMSM_E_NOMEM = -3
SMSM_E_DEVICE = -4
SMSM_E_NUMERIC = -5
SMSM_E_NOT_CONVERGED = -6
SMSM_E_SCRATCH = -7
NOALLOC_SCRATCH_BYTES = 64 << 20
SMSM_FLAG_X_C128 = 0x1
SMSM_FLAG_REG_F32 = 0x2
SMSM_FLAG_GRAM_BF16 = 0x4

# Every entry point of include/smsm.h.
ABI_SYMBOLS = (
    "smsm_plan_create", "smsm_plan_destroy", "smsm_plan_device_bytes", "smsm_workspace_bytes",
    "smsm_set_workspace", "smsm_plan_set_params", "smsm_plan_autotune",
    "smsm_solve", "smsm_solve_noalloc", "smsm_plan_status", "smsm_status_string", "smsm_apply_A", "smsm_apply_AH",
    "smsm_apply_AHA", "smsm_gram", "smsm_weights", "smsm_lambda_max", "smsm_set_weights",
    "smsm_apply_reg", "smsm_apply_normal", "smsm_images_sos", "smsm_launch_kernel", "smsm_kernel_cost",
    "smsm_kernel_timer_start", "smsm_kernel_timer_read", "smsm_batch_create", "smsm_batch_launch",
    "smsm_batch_destroy", "smsm_batch_streams", "smsm_learned_create", "smsm_learned_destroy",
    "smsm_learned_param_count", "smsm_learned_get_params", "smsm_learned_set_params", "smsm_learned_cnn_forward",
    "smsm_learned_cnn_backward", "smsm_learned_solve", "smsm_learned_gradients", "smsm_learned_train_step",
    "smsm_learned_residual", "smsm_learned_solve_fallback", "smsm_learned_set_bf16",
    "smsm_al_create", "smsm_al_destroy", "smsm_al_device_bytes", "smsm_al_solve", "smsm_al_dual",
    "smsm_al_dual_stride",
)
KERNEL_IDS = {"col_normal": 0, "rows_inv": 1, "rows_fwd": 2, "band_corr": 3, "cg_update": 4, "band_extract": 5}


class Geometry(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("n_shots", ctypes.c_int32), ("n_coils", ctypes.c_int32), ("filt", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("n_irls", ctypes.c_int32), ("n_cg", ctypes.c_int32),
                ("eps_frac", ctypes.c_double), ("eps_decay", ctypes.c_double),
                ("eps_floor_frac", ctypes.c_double), ("ns_max_iter", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class ALParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("beta", ctypes.c_double), ("n_outer", ctypes.c_int32),
                ("n_cg", ctypes.c_int32), ("n_sign", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class SmsmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsmsm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1901_01893_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, st = ctypes.c_void_p, ctypes.c_int
        L.smsm_plan_create.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Params), vp,
                                       ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_double),
                                       vp, ctypes.POINTER(vp)]
        L.smsm_plan_create.restype = st
        L.smsm_plan_destroy.argtypes = [vp]
        L.smsm_plan_destroy.restype = st
        L.smsm_plan_device_bytes.argtypes = [vp]
        L.smsm_plan_device_bytes.restype = ctypes.c_size_t
        L.smsm_workspace_bytes.argtypes = [vp]
        L.smsm_workspace_bytes.restype = ctypes.c_size_t
        L.smsm_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.smsm_set_workspace.restype = st
        L.smsm_plan_set_params.argtypes = [vp, ctypes.POINTER(Params)]
        L.smsm_plan_set_params.restype = st
        L.smsm_plan_autotune.argtypes = [vp, st, ctypes.POINTER(ctypes.c_int), vp]
        L.smsm_plan_autotune.restype = st
        L.smsm_solve.argtypes = [vp, vp, vp, vp]
        L.smsm_solve.restype = st
        L.smsm_solve_noalloc.argtypes = [vp, vp, vp, vp]
        L.smsm_solve_noalloc.restype = st
        L.smsm_plan_status.argtypes = [vp]
        L.smsm_plan_status.restype = st
        L.smsm_status_string.argtypes = [st]
        L.smsm_status_string.restype = ctypes.c_char_p
        for name in ("smsm_apply_A", "smsm_apply_AH", "smsm_apply_AHA", "smsm_gram", "smsm_lambda_max",
                     "smsm_apply_reg", "smsm_apply_normal", "smsm_images_sos"):
            f = getattr(L, name)
            f.argtypes = [vp, vp, vp, vp]
            f.restype = st
        L.smsm_weights.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp, vp]
        L.smsm_weights.restype = st
        L.smsm_set_weights.argtypes = [vp, vp, vp]
        L.smsm_set_weights.restype = st
        L.smsm_launch_kernel.argtypes = [vp, st, st, vp]
        L.smsm_launch_kernel.restype = st
        L.smsm_kernel_cost.argtypes = [vp, st, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.smsm_kernel_cost.restype = st
        L.smsm_kernel_timer_start.argtypes = [vp, st, st, st]
        L.smsm_kernel_timer_start.restype = st
        L.smsm_kernel_timer_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.smsm_kernel_timer_read.restype = st
        pvp = ctypes.POINTER(vp)
        L.smsm_batch_create.argtypes = [pvp, st, pvp, pvp, st, pvp]
        L.smsm_batch_create.restype = st
        L.smsm_batch_launch.argtypes = [vp, vp]
        L.smsm_batch_launch.restype = st
        L.smsm_batch_destroy.argtypes = [vp]
        L.smsm_batch_destroy.restype = st
        L.smsm_batch_streams.argtypes = [vp]
        L.smsm_batch_streams.restype = st
        pf, pd = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        L.smsm_learned_create.argtypes = [vp, st, st, st, ctypes.c_double, pf, pvp]
        L.smsm_learned_destroy.argtypes = [vp]
        L.smsm_learned_param_count.argtypes = [vp]
        L.smsm_learned_param_count.restype = ctypes.c_long
        L.smsm_learned_get_params.argtypes = [vp, pf]
        L.smsm_learned_set_params.argtypes = [vp, pf]
        L.smsm_learned_cnn_forward.argtypes = [vp, vp, vp, vp]
        L.smsm_learned_cnn_backward.argtypes = [vp, vp, vp, vp, pf, vp]
        L.smsm_learned_solve.argtypes = [vp, vp, vp, vp]
        L.smsm_learned_gradients.argtypes = [vp, vp, vp, pd, pf, vp]
        L.smsm_learned_train_step.argtypes = [vp, vp, vp, ctypes.c_double, pd, vp]
        L.smsm_learned_residual.argtypes = [vp, vp, vp, pd, vp]
        L.smsm_learned_solve_fallback.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, pd,
                                                  ctypes.POINTER(ctypes.c_int), vp]
        L.smsm_learned_set_bf16.argtypes = [vp, st]
        for name in ("smsm_learned_create", "smsm_learned_destroy", "smsm_learned_get_params",
                     "smsm_learned_set_params", "smsm_learned_cnn_forward", "smsm_learned_cnn_backward",
                     "smsm_learned_solve", "smsm_learned_gradients", "smsm_learned_train_step",
                     "smsm_learned_residual", "smsm_learned_solve_fallback", "smsm_learned_set_bf16"):
            getattr(L, name).restype = st
        L.smsm_al_create.argtypes = [vp, ctypes.POINTER(ALParams), pvp]
        L.smsm_al_create.restype = st
        L.smsm_al_destroy.argtypes = [vp]
        L.smsm_al_destroy.restype = st
        L.smsm_al_device_bytes.argtypes = [vp]
        L.smsm_al_device_bytes.restype = ctypes.c_size_t
        L.smsm_al_solve.argtypes = [vp, vp, vp, vp]
        L.smsm_al_solve.restype = st
        L.smsm_al_dual.argtypes = [vp, vp, vp]
        L.smsm_al_dual.restype = st
        L.smsm_al_dual_stride.argtypes = [vp]
        L.smsm_al_dual_stride.restype = ctypes.c_long
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().smsm_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != SMSM_OK:
        raise SmsmError(status, where)


def _dev_ptr(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_params(lam=1e-3, n_irls=10, n_cg=10, eps_frac=0.1, eps_decay=1.5, eps_floor_frac=1e-4,
                ns_max_iter=0, flags=0) -> Params:
    return Params(float(lam), int(n_irls), int(n_cg), float(eps_frac), float(eps_decay),
                  float(eps_floor_frac), int(ns_max_iter), int(flags))


class Plan:
    """A solver plan for one geometry (wraps smsm_plan_create / destroy).

    workspace: "auto" allocates a torch uint8 tensor of workspace_bytes() on
    the coils' device and binds it (smsm_set_workspace); None leaves the plan
    without one (bind it later with set_workspace)."""

    def __init__(self, n1: int, n2: int, n_slices: int, n_shots: int, n_coils: int, filt: int,
                 coils, masks: np.ndarray, shifts: Optional[Sequence[float]] = None,
                 params: Optional[Params] = None, stream=None, workspace="auto"):
        import torch
        self.geom = Geometry(n1, n2, n_slices, n_shots, n_coils, filt)
        self.params = params if params is not None else make_params()
        self.shape_x = (n_slices, n_shots, n2, n1)
        self.shape_y = (n_shots, n_coils, n2, n1)
        self.K = n_shots * filt * filt
        self.shape_g = (n_slices, self.K, self.K)
        cptr = _dev_ptr(coils, torch.complex64, (n_slices, n_coils, n2, n1), "coils")
        m = np.ascontiguousarray(masks, dtype=np.uint8)
        if m.shape != (n_shots, n2):
            raise ValueError(f"masks: expected {(n_shots, n2)}, got {m.shape}")
        sh = None
        if shifts is not None:
            sh = np.ascontiguousarray(shifts, dtype=np.float64)
            if sh.shape != (n_slices,):
                raise ValueError("shifts: one value per slice")
        self._masks, self._shifts = m, sh
        out = ctypes.c_void_p()
        st = lib().smsm_plan_create(
            ctypes.byref(self.geom), ctypes.byref(self.params), cptr,
            m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
            sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if sh is not None else None,
            _stream_ptr(stream), ctypes.byref(out))
        _check(st, "smsm_plan_create")
        self._h = out
        self._ws = None
        self.device = coils.device
        if isinstance(workspace, str) and workspace == "auto":
            self.set_workspace(torch.empty(self.workspace_bytes(), dtype=torch.uint8, device=coils.device))
        elif workspace is not None:
            self.set_workspace(workspace)

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().smsm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def device_bytes(self) -> int:
        """Device memory the plan holds (not counting its workspace)."""
        return int(lib().smsm_plan_device_bytes(self._h))

    def workspace_bytes(self) -> int:
        return int(lib().smsm_workspace_bytes(self._h))

    def set_workspace(self, ws):
        """Bind a contiguous device tensor of at least workspace_bytes() bytes
        (kept referenced here while bound); None unbinds."""
        if ws is None:
            _check(lib().smsm_set_workspace(self._h, None, 0), "smsm_set_workspace")
            self._ws = None
            return
        if not ws.is_cuda or not ws.is_contiguous():
            raise ValueError("workspace: a contiguous device tensor")
        nbytes = ws.numel() * ws.element_size()
        _check(lib().smsm_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr()), nbytes), "smsm_set_workspace")
        self._ws = ws

    def set_params(self, params: Params):
        _check(lib().smsm_plan_set_params(self._h, ctypes.byref(params)), "smsm_plan_set_params")
        self.params = params

    def autotune(self, reps: int = 20, stream=None):
        """Choose the launch shapes by timing (smsm_plan_autotune); returns
        (rows per workgroup of the row transforms, columns per wave of the
        vector pass)."""
        shape = (ctypes.c_int * 2)()
        _check(lib().smsm_plan_autotune(self._h, int(reps), shape, _stream_ptr(stream)), "smsm_plan_autotune")
        return shape[0], shape[1]

    # -- solve ----------------------------------------------------------------
    def solve(self, y, out=None, stream=None):
        """x = IRLS solve of Eq. 10 for y (c64 [Ns][Nc][n2][n1])."""
        import torch
        c128 = bool(self.params.flags & SMSM_FLAG_X_C128)
        dt = torch.complex128 if c128 else torch.complex64
        if out is None:
            out = torch.empty(self.shape_x, dtype=dt, device=y.device)
        yp = _dev_ptr(y, torch.complex64, self.shape_y, "y")
        xp = _dev_ptr(out, dt, self.shape_x, "x")
        _check(lib().smsm_solve(self._h, yp, xp, _stream_ptr(stream)), "smsm_solve")
        return out

    def solve_noalloc(self, y, out, stream=None):
        """The same solve run in the library's static device scratch (no
        allocation anywhere; `out` must be given).  Calls that overlap on one
        device race."""
        import torch
        c128 = bool(self.params.flags & SMSM_FLAG_X_C128)
        dt = torch.complex128 if c128 else torch.complex64
        yp = _dev_ptr(y, torch.complex64, self.shape_y, "y")
        xp = _dev_ptr(out, dt, self.shape_x, "x")
        _check(lib().smsm_solve_noalloc(self._h, yp, xp, _stream_ptr(stream)), "smsm_solve_noalloc")
        return out

    def status(self) -> int:
        return int(lib().smsm_plan_status(self._h))

    # -- operators --------------------------------------------------------------
    def _unary(self, fname, a, a_dtype, a_shape, out_shape, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(out_shape, dtype=torch.complex128, device=a.device)
        ap = _dev_ptr(a, a_dtype, a_shape, "input")
        op = _dev_ptr(out, torch.complex128, out_shape, "output")
        _check(getattr(lib(), fname)(self._h, ap, op, _stream_ptr(stream)), fname)
        return out

    def apply_A(self, x, out=None, stream=None):
        import torch
        return self._unary("smsm_apply_A", x, torch.complex128, self.shape_x, self.shape_y, out, stream)

    def apply_AH(self, y, out=None, stream=None):
        import torch
        return self._unary("smsm_apply_AH", y, torch.complex64, self.shape_y, self.shape_x, out, stream)

    def apply_AHA(self, x, out=None, stream=None):
        import torch
        return self._unary("smsm_apply_AHA", x, torch.complex128, self.shape_x, self.shape_x, out, stream)

    def gram(self, x, out=None, stream=None):
        import torch
        return self._unary("smsm_gram", x, torch.complex128, self.shape_x, self.shape_g, out, stream)

    def apply_reg(self, x, out=None, stream=None):
        import torch
        return self._unary("smsm_apply_reg", x, torch.complex128, self.shape_x, self.shape_x, out, stream)

    def apply_normal(self, x, out=None, stream=None):
        import torch
        return self._unary("smsm_apply_normal", x, torch.complex128, self.shape_x, self.shape_x, out, stream)

    def images_sos(self, x, out=None, stream=None):
        """Root-sum-of-squares image per slice of k-space x (c128 [L][Ns][n2][n1]) -> float64 [L][n2][n1]."""
        import torch
        shape = (self.geom.n_slices, self.geom.n2, self.geom.n1)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=x.device)
        xp = _dev_ptr(x, torch.complex128, self.shape_x, "x")
        op = _dev_ptr(out, torch.float64, shape, "img")
        _check(lib().smsm_images_sos(self._h, xp, op, _stream_ptr(stream)), "smsm_images_sos")
        return out

    def lambda_max(self, G, stream=None):
        import torch
        out = torch.empty(self.geom.n_slices, dtype=torch.float64, device=G.device)
        gp = _dev_ptr(G, torch.complex128, self.shape_g, "G")
        _check(lib().smsm_lambda_max(self._h, gp, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "smsm_lambda_max")
        return out

    def weights(self, G, eps: Sequence[float], out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape_g, dtype=torch.complex128, device=G.device)
        e = np.ascontiguousarray(eps, dtype=np.float64)
        if e.shape != (self.geom.n_slices,):
            raise ValueError("eps: one value per slice")
        gp = _dev_ptr(G, torch.complex128, self.shape_g, "G")
        wp = _dev_ptr(out, torch.complex128, self.shape_g, "W")
        _check(lib().smsm_weights(self._h, gp, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), wp,
                                  _stream_ptr(stream)), "smsm_weights")
        return out

    def set_weights(self, W, stream=None):
        import torch
        wp = _dev_ptr(W, torch.complex128, self.shape_g, "W")
        _check(lib().smsm_set_weights(self._h, wp, _stream_ptr(stream)), "smsm_set_weights")


    # -- diagnostics -------------------------------------------------------------
    def launch_kernel(self, name: str, reps: int = 1, stream=None):
        """Re-launch one CG-iteration kernel `reps` times on the plan's buffers."""
        _check(lib().smsm_launch_kernel(self._h, KERNEL_IDS[name], int(reps), _stream_ptr(stream)),
               "smsm_launch_kernel")

    def kernel_timer_start(self, name: str, capacity: int, stride: int = 1):
        """Time (start/stop events per dispatch) one launch of a kernel in every `stride`, up to
        `capacity` of them; capacity 0 turns it off."""
        _check(lib().smsm_kernel_timer_start(self._h, KERNEL_IDS[name], int(capacity), int(stride)),
               "smsm_kernel_timer_start")

    def kernel_timer_read(self):
        """(summed milliseconds, launches) of the timed launches since the start or the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        _check(lib().smsm_kernel_timer_read(self._h, ctypes.byref(ms), ctypes.byref(n)), "smsm_kernel_timer_read")
        return ms.value, n.value

    def kernel_cost(self, name: str):
        """(FP64 flops, compulsory HBM bytes) of one launch of a CG-iteration kernel."""
        f, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().smsm_kernel_cost(self._h, KERNEL_IDS[name], ctypes.byref(f), ctypes.byref(b)),
               "smsm_kernel_cost")
        return f.value, b.value


# Flat names mirroring the C ABI: each is the marshalling method itself, taking
# the plan first (smsm_solve(plan, y) is plan.solve(y)).
smsm_plan_create = Plan
smsm_plan_destroy = Plan.close
smsm_plan_device_bytes = Plan.device_bytes
smsm_workspace_bytes = Plan.workspace_bytes
smsm_set_workspace = Plan.set_workspace
smsm_plan_set_params = Plan.set_params
smsm_plan_autotune = Plan.autotune
smsm_solve = Plan.solve
smsm_solve_noalloc = Plan.solve_noalloc
smsm_plan_status = Plan.status
smsm_apply_A = Plan.apply_A
smsm_apply_AH = Plan.apply_AH
smsm_apply_AHA = Plan.apply_AHA
smsm_gram = Plan.gram
smsm_weights = Plan.weights
smsm_lambda_max = Plan.lambda_max
smsm_set_weights = Plan.set_weights
smsm_apply_reg = Plan.apply_reg
smsm_apply_normal = Plan.apply_normal
smsm_images_sos = Plan.images_sos
smsm_launch_kernel = Plan.launch_kernel
smsm_kernel_cost = Plan.kernel_cost
smsm_kernel_timer_start = Plan.kernel_timer_start
smsm_kernel_timer_read = Plan.kernel_timer_read
smsm_status_string = status_string


class Batch:
    """Solves of several plans captured as one graph on concurrent streams
    (smsm_batch_*): launch() runs x_k = solve(plan_k, y_k) for every k.  The
    tensors are baked in: refill ys in place before a launch."""

    def __init__(self, plans, ys, xs, n_streams: int = 2):
        """n_streams = 0 lets the library pick the stream count by timing the candidates."""
        import torch
        n = len(plans)
        if not (len(ys) == len(xs) == n):
            raise ValueError("one y and one x per plan")
        yp, xp = [], []
        for pl, y, x in zip(plans, ys, xs):
            c128 = bool(pl.params.flags & SMSM_FLAG_X_C128)
            yp.append(_dev_ptr(y, torch.complex64, pl.shape_y, "y").value)
            xp.append(_dev_ptr(x, torch.complex128 if c128 else torch.complex64, pl.shape_x, "x").value)
        arr = ctypes.c_void_p * n
        h = ctypes.c_void_p()
        _check(lib().smsm_batch_create(arr(*[pl._h for pl in plans]), n, arr(*yp), arr(*xp), int(n_streams),
                                       ctypes.byref(h)), "smsm_batch_create")
        self._h = h
        self._keep = (list(plans), list(ys), list(xs))

    def launch(self, stream=None):
        _check(lib().smsm_batch_launch(self._h, _stream_ptr(stream)), "smsm_batch_launch")

    @property
    def n_streams(self) -> int:
        return int(lib().smsm_batch_streams(self._h))

    def close(self):
        if self._h is not None:
            lib().smsm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


smsm_batch_create = Batch
smsm_batch_launch = Batch.launch
smsm_batch_destroy = Batch.close
smsm_batch_streams = Batch.n_streams.fget


def flatten_params(params) -> "np.ndarray":
    """[(w [co][ci][3][3], b [co]), ...] -> the flat float32 layout of the C ABI."""
    return np.concatenate([np.concatenate([np.asarray(w, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                           for w, b in params]).astype(np.float32)


def unflatten_params(flat, c_io: int, width: int, depth: int = 5) -> list:
    chans = [c_io] + [width] * (depth - 1) + [c_io]
    out, off = [], 0
    for k in range(depth):
        ci, co = chans[k], chans[k + 1]
        w = flat[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = flat[off:off + co]
        off += co
        out.append((w, b))
    return out


class Learned:
    """The learned unrolled solver on a plan (smsm_learned_*): a residual CNN
    prior over each slice's 2 Ns k-space channels inside n_unroll
    data-consistency iterations."""

    def __init__(self, plan: Plan, params, width: int = 64, n_unroll: int = 5, n_cg: int = 10, mu: float = 1.0):
        flat = flatten_params(params)
        h = ctypes.c_void_p()
        _check(lib().smsm_learned_create(plan._h, int(width), int(n_unroll), int(n_cg), float(mu),
                                         flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h)),
               "smsm_learned_create")
        self._h = h
        self.plan = plan
        self.width, self.n_unroll, self.n_cg, self.mu = width, n_unroll, n_cg, mu
        self.c_io = 2 * plan.shape_x[1]
        self.shape_c = (plan.shape_x[0], self.c_io, plan.shape_x[2], plan.shape_x[3])

    def param_count(self) -> int:
        return int(lib().smsm_learned_param_count(self._h))

    def get_params(self) -> "np.ndarray":
        out = np.empty(self.param_count(), np.float32)
        _check(lib().smsm_learned_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "smsm_learned_get_params")
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, np.float32)
        _check(lib().smsm_learned_set_params(self._h, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "smsm_learned_set_params")

    def set_bf16(self, mode: int = 1):
        """0: FP32 weights; 1: BF16 weights, exact products; 2: the BF16
        network (convolution inputs rounded to BF16 too).  True means 1."""
        _check(lib().smsm_learned_set_bf16(self._h, int(mode)), "smsm_learned_set_bf16")

    def cnn_forward(self, inp, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape_c, dtype=torch.float32, device=inp.device)
        _check(lib().smsm_learned_cnn_forward(self._h, _dev_ptr(inp, torch.float32, self.shape_c, "in"),
                                              _dev_ptr(out, torch.float32, self.shape_c, "out"),
                                              _stream_ptr(stream)), "smsm_learned_cnn_forward")
        return out

    def cnn_backward(self, inp, gout, stream=None):
        import torch
        gin = torch.empty(self.shape_c, dtype=torch.float32, device=inp.device)
        grads = np.empty(self.param_count(), np.float32)
        _check(lib().smsm_learned_cnn_backward(self._h, _dev_ptr(inp, torch.float32, self.shape_c, "in"),
                                               _dev_ptr(gout, torch.float32, self.shape_c, "gout"),
                                               _dev_ptr(gin, torch.float32, self.shape_c, "gin"),
                                               grads.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                               _stream_ptr(stream)), "smsm_learned_cnn_backward")
        return gin, grads

    def solve(self, y, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.plan.shape_x, dtype=torch.complex128, device=y.device)
        _check(lib().smsm_learned_solve(self._h, _dev_ptr(y, torch.complex64, self.plan.shape_y, "y"),
                                        _dev_ptr(out, torch.complex128, self.plan.shape_x, "x"),
                                        _stream_ptr(stream)), "smsm_learned_solve")
        return out

    def gradients(self, y, xt, stream=None):
        import torch
        loss = ctypes.c_double()
        grads = np.empty(self.param_count(), np.float32)
        _check(lib().smsm_learned_gradients(self._h, _dev_ptr(y, torch.complex64, self.plan.shape_y, "y"),
                                            _dev_ptr(xt, torch.complex128, self.plan.shape_x, "xt"),
                                            ctypes.byref(loss), grads.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            _stream_ptr(stream)), "smsm_learned_gradients")
        return loss.value, grads

    def train_step(self, y, xt, lr: float, stream=None) -> float:
        import torch
        loss = ctypes.c_double()
        _check(lib().smsm_learned_train_step(self._h, _dev_ptr(y, torch.complex64, self.plan.shape_y, "y"),
                                             _dev_ptr(xt, torch.complex128, self.plan.shape_x, "xt"),
                                             float(lr), ctypes.byref(loss), _stream_ptr(stream)),
               "smsm_learned_train_step")
        return loss.value

    def residual(self, x, y, stream=None) -> float:
        import torch
        r = ctypes.c_double()
        _check(lib().smsm_learned_residual(self._h, _dev_ptr(x, torch.complex128, self.plan.shape_x, "x"),
                                           _dev_ptr(y, torch.complex64, self.plan.shape_y, "y"), ctypes.byref(r),
                                           _stream_ptr(stream)), "smsm_learned_residual")
        return r.value

    def solve_fallback(self, y, ratio: float = 1.5, res_ref: float = 0.0, out=None, stream=None):
        """The learned solve, replaced by the plain IRLS solve when its
        data-consistency residual exceeds ratio x the reference (res_ref, or
        the plain solve's own when res_ref <= 0).  Returns (x, fell_back,
        learned residual, reference residual)."""
        import torch
        if out is None:
            out = torch.empty(self.plan.shape_x, dtype=torch.complex128, device=y.device)
        res = (ctypes.c_double * 2)()
        fb = ctypes.c_int()
        _check(lib().smsm_learned_solve_fallback(self._h, _dev_ptr(y, torch.complex64, self.plan.shape_y, "y"),
                                                 _dev_ptr(out, torch.complex128, self.plan.shape_x, "x"),
                                                 float(ratio), float(res_ref), res, ctypes.byref(fb),
                                                 _stream_ptr(stream)), "smsm_learned_solve_fallback")
        return out, bool(fb.value), res[0], res[1]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().smsm_learned_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


smsm_learned_create = Learned
smsm_learned_destroy = Learned.close
smsm_learned_param_count = Learned.param_count
smsm_learned_get_params = Learned.get_params
smsm_learned_set_params = Learned.set_params
smsm_learned_cnn_forward = Learned.cnn_forward
smsm_learned_cnn_backward = Learned.cnn_backward
smsm_learned_solve = Learned.solve
smsm_learned_gradients = Learned.gradients
smsm_learned_train_step = Learned.train_step
smsm_learned_residual = Learned.residual
smsm_learned_solve_fallback = Learned.solve_fallback
smsm_learned_set_bf16 = Learned.set_bf16


class AL:
    """The augmented-Lagrangian solve of Eq. 10 on a plan (smsm_al_*): the
    split Z = H(x) with scaled duals U, singular-value thresholding at
    lam / beta, n_outer outer iterations of n_cg CG steps each."""

    def __init__(self, plan: Plan, lam: float, beta: float, n_outer: int = 30, n_cg: int = 5, n_sign: int = 0,
                 c128: bool = True):
        p = ALParams(float(lam), float(beta), int(n_outer), int(n_cg), int(n_sign),
                     SMSM_FLAG_X_C128 if c128 else 0)
        h = ctypes.c_void_p()
        _check(lib().smsm_al_create(plan._h, ctypes.byref(p), ctypes.byref(h)), "smsm_al_create")
        self._h = h
        self.plan = plan
        self.lam, self.beta, self.n_outer, self.n_cg, self.c128 = lam, beta, n_outer, n_cg, c128
        L, Ns, n2, n1 = plan.shape_x
        r = plan.geom.filt
        self.n_anchor = (n2 - r + 1) * (n1 - r + 1)
        self.shape_dual = (L, Ns * r * r, int(lib().smsm_al_dual_stride(h)))

    def device_bytes(self) -> int:
        return int(lib().smsm_al_device_bytes(self._h))

    def solve(self, y, out=None, stream=None):
        import torch
        dt = torch.complex128 if self.c128 else torch.complex64
        if out is None:
            out = torch.empty(self.plan.shape_x, dtype=dt, device=y.device)
        _check(lib().smsm_al_solve(self._h, _dev_ptr(y, torch.complex64, self.plan.shape_y, "y"),
                                   _dev_ptr(out, dt, self.plan.shape_x, "x"), _stream_ptr(stream)), "smsm_al_solve")
        return out

    def dual(self, out=None, stream=None):
        """The scaled duals of the last solve, [L][K][stride] complex128
        (entry [l][k][p] = U_l[p][k] for p < n_anchor, zero beyond)."""
        import torch
        if out is None:
            out = torch.empty(self.shape_dual, dtype=torch.complex128, device=self.plan.device)
        _check(lib().smsm_al_dual(self._h, _dev_ptr(out, torch.complex128, self.shape_dual, "u"),
                                  _stream_ptr(stream)), "smsm_al_dual")
        return out

    def dual_stride(self) -> int:
        return int(lib().smsm_al_dual_stride(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().smsm_al_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


smsm_al_create = AL
smsm_al_destroy = AL.close
smsm_al_device_bytes = AL.device_bytes
smsm_al_solve = AL.solve
smsm_al_dual = AL.dual
smsm_al_dual_stride = AL.dual_stride
