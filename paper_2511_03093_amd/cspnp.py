"""ctypes binding of libcspnp (include/cspnp.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  The functions named ``cspnp_*`` mirror the C entry points one to
one and take raw addresses; :class:`Plan` wraps them for torch tensors on the
current HIP stream (torch supplies device memory and streams, nothing else).
Importing this module never computes anything; :func:`load` raises when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcspnp.so")

OK, EINVAL, ENOMEM, EHIP, ENODEV, EUNSUPPORTED, ENONFINITE = range(7)
ZBC = {"periodic": 0, "neumann": 1}
DENOISER = {"tikhonov": 0, "tv": 1, "bm3d": 2}
FLAG_NO_GRAPH = 1
FLAG_CHECK_FINITE = 2
FLAG_PAPER_SCHEDULE = 4
WS_SOLVE, WS_DENOISE, WS_SOLVE_TOL = 0, 1, 2


class Desc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("R", ctypes.c_int32),
                ("N", ctypes.c_int32), ("zbc", ctypes.c_int32), ("denoiser", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("rho", ctypes.c_double), ("gamma", ctypes.c_double),
                ("iters", ctypes.c_int32), ("tv_inner", ctypes.c_int32), ("tv_tau", ctypes.c_double),
                ("bm3d_sigma", ctypes.c_double), ("flags", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tv_shape", ctypes.c_int32), ("xu_block", ctypes.c_int32)]


class CspnpError(RuntimeError):
    def __init__(self, status, func, detail):
        self.status = status
        super().__init__(f"{func} -> {status}: {detail}")


_P = ctypes.c_void_p
_SIGNATURES = {
    "cspnp_version": ([], ctypes.c_int),
    "cspnp_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "cspnp_last_error": ([], ctypes.c_char_p),
    "cspnp_plan_create": ([ctypes.POINTER(Desc), _P, ctypes.c_int, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "cspnp_plan_destroy": ([_P], ctypes.c_int),
    "cspnp_plan_desc": ([_P, ctypes.POINTER(Desc)], ctypes.c_int),
    "cspnp_workspace_size": ([_P, ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "cspnp_forward": ([_P, _P, _P, _P], ctypes.c_int),
    "cspnp_adjoint": ([_P, _P, _P, _P], ctypes.c_int),
    "cspnp_xupdate": ([_P, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "cspnp_denoise": ([_P, ctypes.POINTER(Params), _P, _P, _P, _P, _P], ctypes.c_int),
    "cspnp_solve": ([_P, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "cspnp_tuning_candidates": ([ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "cspnp_tv_shape_info": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "cspnp_plan_get_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int),
    "cspnp_plan_set_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int),
    "cspnp_autotune": ([_P, ctypes.POINTER(Params), ctypes.c_char_p, ctypes.c_int, _P], ctypes.c_int),
    "cspnp_ckpt_size": ([_P, ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "cspnp_bwd_workspace_size": ([_P, ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                                 ctypes.c_int),
    "cspnp_solve_ckpt": ([_P, ctypes.POINTER(Params), _P, _P, _P, _P, ctypes.c_int, _P, _P, _P], ctypes.c_int),
    "cspnp_solve_bwd": ([_P, ctypes.POINTER(Params), _P, ctypes.c_int, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "cspnp_solve_tol": ([_P, ctypes.POINTER(Params), ctypes.c_double, ctypes.c_int, _P, _P, _P, _P, _P, _P,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "cspnp_metrics_workspace_size": ([ctypes.c_int32] * 4 + [ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "cspnp_psnr": ([_P, _P, ctypes.c_size_t, ctypes.c_double, _P, _P, _P], ctypes.c_int),
    "cspnp_ssim": ([_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P, _P,
                    _P], ctypes.c_int),
    "cspnp_rel_change": ([_P, _P, ctypes.c_size_t, _P, _P, _P], ctypes.c_int),
    "cspnp_bm3d_stage": ([_P, ctypes.POINTER(Params), _P, ctypes.c_int, _P, _P], ctypes.c_int),
    "cspnp_bm3d_layout": ([_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                           ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "cspnp_batch_create": ([ctypes.c_int32, ctypes.POINTER(Desc), ctypes.POINTER(_P), _P, ctypes.POINTER(_P)],
                           ctypes.c_int),
    "cspnp_batch_destroy": ([_P], ctypes.c_int),
    "cspnp_batch_workspace_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "cspnp_batch_solve": ([_P, ctypes.POINTER(Params), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                           ctypes.POINTER(_P), _P, _P], ctypes.c_int),
    "cspnp_batch_set_tv_shape": ([_P, ctypes.c_int32], ctypes.c_int),
    "cspnp_batch_get_tv_shape": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "cspnp_batch_autotune": ([_P, ctypes.POINTER(Params), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                              ctypes.POINTER(_P), _P, _P], ctypes.c_int),
}

_lib = None


def declared_symbols():
    """Entry points declared in include/*.h (parsed from the headers)."""
    import re
    inc = os.path.join(os.path.dirname(HERE), "include")
    names = []
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(cspnp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def load(path=LIB_PATH):
    """Load libcspnp.so and declare its entry points; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2511_03093_amd.build (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status, func):
    if status != OK:
        lib = load()
        detail = lib.cspnp_last_error().decode()
        raise CspnpError(status, func, detail)
    return status


def _call(name, *args):
    return check(getattr(load(), name)(*args), name)


def make_params(lam=0.05, rho=1.0, gamma=0.0, iters=1, tv_inner=10, tv_tau=0.125,
                bm3d_sigma=9.669 / 255.0, flags=0, **_ignored):
    return Params(float(lam), float(rho), float(gamma), int(iters), int(tv_inner), float(tv_tau),
                  float(bm3d_sigma), int(flags))


def params_from(p, **over):
    """Params struct from a dict or an object with lam/rho/gamma/... attributes."""
    if not isinstance(p, dict):
        p = {k: getattr(p, k) for k in ("lam", "rho", "gamma", "iters", "tv_inner", "tv_tau", "bm3d_sigma")
             if hasattr(p, k)}
    q = dict(p)
    q.update(over)
    return make_params(**q)


# --- one-to-one wrappers of the C entry points (raw addresses) -------------

def cspnp_version():
    return load().cspnp_version()


def cspnp_status_string(status):
    return load().cspnp_status_string(status).decode()


def cspnp_last_error():
    return load().cspnp_last_error().decode()


def cspnp_plan_create(desc, masks_ptr, masks_on_device, stream):
    out = _P()
    _call("cspnp_plan_create", ctypes.byref(desc), _P(masks_ptr), int(masks_on_device), _P(stream),
          ctypes.byref(out))
    return out


def cspnp_plan_destroy(plan):
    _call("cspnp_plan_destroy", plan)


def cspnp_plan_desc(plan):
    d = Desc()
    _call("cspnp_plan_desc", plan, ctypes.byref(d))
    return d


def cspnp_workspace_size(plan, params, mode):
    n = ctypes.c_size_t()
    _call("cspnp_workspace_size", plan, ctypes.byref(params), int(mode), ctypes.byref(n))
    return n.value


def cspnp_forward(plan, x, y, stream):
    _call("cspnp_forward", plan, _P(x), _P(y), _P(stream))


def cspnp_adjoint(plan, y, x, stream):
    _call("cspnp_adjoint", plan, _P(y), _P(x), _P(stream))


def cspnp_xupdate(plan, params, y, u, d, x_out, f_out, stream):
    _call("cspnp_xupdate", plan, ctypes.byref(params), _P(y), _P(u), _P(d), _P(x_out), _P(f_out), _P(stream))


def cspnp_denoise(plan, params, f, u, d_out, ws, stream):
    _call("cspnp_denoise", plan, ctypes.byref(params), _P(f), _P(u), _P(d_out), _P(ws), _P(stream))


def cspnp_solve(plan, params, y, u, d, x, ws, stream):
    _call("cspnp_solve", plan, ctypes.byref(params), _P(y), _P(u), _P(d), _P(x), _P(ws), _P(stream))


def cspnp_tuning_candidates():
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _call("cspnp_tuning_candidates", ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def cspnp_tv_shape_info(index):
    c, r, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _call("cspnp_tv_shape_info", int(index), ctypes.byref(c), ctypes.byref(r), ctypes.byref(t))
    return c.value, r.value, t.value


def cspnp_plan_get_tuning(plan):
    t = Tuning()
    _call("cspnp_plan_get_tuning", plan, ctypes.byref(t))
    return t.tv_shape, t.xu_block


def cspnp_plan_set_tuning(plan, tv_shape, xu_block):
    t = Tuning(int(tv_shape), int(xu_block))
    _call("cspnp_plan_set_tuning", plan, ctypes.byref(t))


def cspnp_autotune(plan, params, cache_path, force, stream):
    cp = cache_path.encode() if cache_path else None
    _call("cspnp_autotune", plan, ctypes.byref(params), cp, int(force), _P(stream))


def cspnp_ckpt_size(plan, params, ckpt_every):
    n = ctypes.c_size_t()
    _call("cspnp_ckpt_size", plan, ctypes.byref(params), int(ckpt_every), ctypes.byref(n))
    return n.value


def cspnp_bwd_workspace_size(plan, params, ckpt_every):
    n = ctypes.c_size_t()
    _call("cspnp_bwd_workspace_size", plan, ctypes.byref(params), int(ckpt_every), ctypes.byref(n))
    return n.value


def cspnp_solve_ckpt(plan, params, y, u, d, x, ckpt_every, ckpt, ws, stream):
    _call("cspnp_solve_ckpt", plan, ctypes.byref(params), _P(y), _P(u), _P(d), _P(x), int(ckpt_every), _P(ckpt),
          _P(ws), _P(stream))


def cspnp_solve_bwd(plan, params, y, ckpt_every, ckpt, x_bar, y_bar, param_bar, ws, stream):
    _call("cspnp_solve_bwd", plan, ctypes.byref(params), _P(y), int(ckpt_every), _P(ckpt), _P(x_bar), _P(y_bar),
          _P(param_bar), _P(ws), _P(stream))


def cspnp_solve_tol(plan, params, tol, check_every, y, u, d, x, ws, stream):
    it = ctypes.c_int32()
    rel = ctypes.c_double()
    _call("cspnp_solve_tol", plan, ctypes.byref(params), float(tol), int(check_every), _P(y), _P(u), _P(d), _P(x),
          _P(ws), _P(stream), ctypes.byref(it), ctypes.byref(rel))
    return it.value, rel.value


def cspnp_metrics_workspace_size(D, H, W, dims):
    n = ctypes.c_size_t()
    _call("cspnp_metrics_workspace_size", int(D), int(H), int(W), int(dims), ctypes.byref(n))
    return n.value


def cspnp_psnr(est, ref, n, peak, out, ws, stream):
    _call("cspnp_psnr", _P(est), _P(ref), int(n), float(peak), _P(out), _P(ws), _P(stream))


def cspnp_ssim(est, ref, D, H, W, dims, L, out, ws, stream):
    _call("cspnp_ssim", _P(est), _P(ref), int(D), int(H), int(W), int(dims), float(L), _P(out), _P(ws), _P(stream))


def cspnp_rel_change(a, b, n, out, ws, stream):
    _call("cspnp_rel_change", _P(a), _P(b), int(n), _P(out), _P(ws), _P(stream))


def _metric(fn_name, dims, est, ref, *extra):
    """Run one metric on device tensors; returns the Python float."""
    torch = _torch()
    D, H, W = est.shape if est.dim() == 3 else (1, *est.shape[-2:])
    nb = cspnp_metrics_workspace_size(D, H, W, dims)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    wsp = (ws.data_ptr() + 255) & ~255
    if fn_name == "psnr":
        cspnp_psnr(_ptr(est, "est"), _ptr(ref, "ref"), est.numel(), extra[0], out.data_ptr(), wsp, _stream())
    elif fn_name == "ssim":
        cspnp_ssim(_ptr(est, "est"), _ptr(ref, "ref"), D, H, W, dims, extra[0], out.data_ptr(), wsp, _stream())
    else:
        cspnp_rel_change(_ptr(est, "a"), _ptr(ref, "b"), est.numel(), out.data_ptr(), wsp, _stream())
    return float(out.item())


def psnr(est, ref, peak=1.0):
    return _metric("psnr", 0, est, ref, peak)


def ssim(est, ref, dims=2, L=1.0):
    return _metric("ssim", dims, est, ref, L)


def rel_change(a, b):
    return _metric("rel", 0, a, b)


def cspnp_bm3d_stage(plan, params, f, stage, ws, stream):
    _call("cspnp_bm3d_stage", plan, ctypes.byref(params), _P(f), int(stage), _P(ws), _P(stream))


def cspnp_bm3d_layout(plan):
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    ny, nx = ctypes.c_int32(), ctypes.c_int32()
    _call("cspnp_bm3d_layout", plan, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(ny),
          ctypes.byref(nx))
    return dict(matches=a.value, counts=b.value, basic=c.value, nry=ny.value, nrx=nx.value)


def _ptr_array(ptrs):
    return (_P * len(ptrs))(*[_P(p) for p in ptrs])


def cspnp_batch_create(descs, mask_ptrs, stream):
    out = _P()
    arr = (Desc * len(descs))(*descs)
    _call("cspnp_batch_create", len(descs), arr, _ptr_array(mask_ptrs), _P(stream), ctypes.byref(out))
    return out


def cspnp_batch_destroy(batch):
    _call("cspnp_batch_destroy", batch)


def cspnp_batch_workspace_size(batch):
    n = ctypes.c_size_t()
    _call("cspnp_batch_workspace_size", batch, ctypes.byref(n))
    return n.value


def cspnp_batch_solve(batch, params_list, y, u, d, x, ws, stream):
    arr = (Params * len(params_list))(*params_list)
    _call("cspnp_batch_solve", batch, arr, _ptr_array(y), _ptr_array(u), _ptr_array(d), _ptr_array(x), _P(ws),
          _P(stream))


def cspnp_batch_set_tv_shape(batch, shape):
    _call("cspnp_batch_set_tv_shape", batch, int(shape))


def cspnp_batch_get_tv_shape(batch):
    s = ctypes.c_int32()
    _call("cspnp_batch_get_tv_shape", batch, ctypes.byref(s))
    return s.value


def cspnp_batch_autotune(batch, params_list, y, u, d, x, ws, stream):
    arr = (Params * len(params_list))(*params_list)
    _call("cspnp_batch_autotune", batch, arr, _ptr_array(y), _ptr_array(u), _ptr_array(d), _ptr_array(x), _P(ws),
          _P(stream))


# --- torch-tensor convenience layer -----------------------------------------

def _torch():
    import torch
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _ptr(t, name, shape=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


class Plan:
    """A problem shape plus packed masks on the current device."""

    def __init__(self, masks, N=1, zbc="periodic", denoiser="tv"):
        torch = _torch()
        if isinstance(masks, torch.Tensor):
            m = masks.to(torch.uint8).contiguous()
        else:
            import numpy as np
            m = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint8))
        R, H, W = m.shape
        self.desc = Desc(H, W, R, N, ZBC[zbc], DENOISER[denoiser])
        self.H, self.W, self.R, self.N = H, W, R, N
        self.zbc, self.denoiser = zbc, denoiser
        self._handle = None
        on_dev = 1 if m.is_cuda else 0
        self._handle = cspnp_plan_create(self.desc, m.data_ptr(), on_dev, _stream())

    @property
    def vol_shape(self):
        return (self.N * self.R, self.H, self.W)

    @property
    def frame_shape(self):
        return (self.N, self.H, self.W)

    def close(self):
        if self._handle is not None:
            cspnp_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, shape):
        torch = _torch()
        return torch.empty(shape, dtype=torch.float32, device="cuda")

    def workspace(self, params, mode=WS_SOLVE):
        torch = _torch()
        n = cspnp_workspace_size(self._handle, params, mode)
        if n == 0:
            return None
        return torch.empty(n + 256, dtype=torch.uint8, device="cuda")

    @staticmethod
    def _ws_ptr(ws):
        if ws is None:
            return None
        p = ws.data_ptr()
        return (p + 255) & ~255

    def forward(self, x, y=None):
        y = self._empty(self.frame_shape) if y is None else y
        cspnp_forward(self._handle, _ptr(x, "x", self.vol_shape), _ptr(y, "y", self.frame_shape), _stream())
        return y

    def adjoint(self, y, x=None):
        x = self._empty(self.vol_shape) if x is None else x
        cspnp_adjoint(self._handle, _ptr(y, "y", self.frame_shape), _ptr(x, "x", self.vol_shape), _stream())
        return x

    def xupdate(self, params, y, u, d, want_x=True, want_f=True):
        x = self._empty(self.vol_shape) if want_x else None
        f = self._empty(self.vol_shape) if want_f else None
        cspnp_xupdate(self._handle, params, _ptr(y, "y", self.frame_shape), _ptr(u, "u", self.vol_shape),
                      _ptr(d, "d", self.vol_shape), _ptr(x, "x_out") if x is not None else None,
                      _ptr(f, "f_out") if f is not None else None, _stream())
        return x, f

    def denoise(self, params, f, want_d=True, ws=None):
        u = self._empty(self.vol_shape)
        d = self._empty(self.vol_shape) if want_d else None
        ws = self.workspace(params, WS_DENOISE) if ws is None else ws
        cspnp_denoise(self._handle, params, _ptr(f, "f", self.vol_shape), _ptr(u, "u"),
                      _ptr(d, "d_out") if d is not None else None, self._ws_ptr(ws), _stream())
        return u, d

    def tuning(self):
        return cspnp_plan_get_tuning(self._handle)

    def set_tuning(self, tv_shape, xu_block):
        cspnp_plan_set_tuning(self._handle, tv_shape, xu_block)

    def autotune(self, params, cache_path=None, force=False):
        cspnp_autotune(self._handle, params, cache_path, force, _stream())
        return self.tuning()

    def solve_tol(self, params, y, tol, check_every=1, u=None, d=None, x=None):
        """Iterate until the relative change of x drops below tol (at most params.iters); returns
        (x, u, d, iterations, last relative change)."""
        torch = _torch()
        u = torch.zeros(self.vol_shape, dtype=torch.float32, device="cuda") if u is None else u
        d = torch.zeros(self.vol_shape, dtype=torch.float32, device="cuda") if d is None else d
        x = self._empty(self.vol_shape) if x is None else x
        ws = self.workspace(params, WS_SOLVE_TOL)
        it, rel = cspnp_solve_tol(self._handle, params, tol, check_every, _ptr(y, "y", self.frame_shape),
                                  _ptr(u, "u", self.vol_shape), _ptr(d, "d", self.vol_shape),
                                  _ptr(x, "x", self.vol_shape), self._ws_ptr(ws), _stream())
        return x, u, d, it, rel

    def solve(self, params, y, u=None, d=None, x=None, ws=None):
        """Run params.iters iterations in place on (u, d); returns (x, u, d)."""
        torch = _torch()
        u = torch.zeros(self.vol_shape, dtype=torch.float32, device="cuda") if u is None else u
        d = torch.zeros(self.vol_shape, dtype=torch.float32, device="cuda") if d is None else d
        x = self._empty(self.vol_shape) if x is None else x
        ws = self.workspace(params, WS_SOLVE) if ws is None else ws
        cspnp_solve(self._handle, params, _ptr(y, "y", self.frame_shape), _ptr(u, "u", self.vol_shape),
                    _ptr(d, "d", self.vol_shape), _ptr(x, "x", self.vol_shape), self._ws_ptr(ws), _stream())
        return x, u, d


class Batch:
    """Many independent snapshots solved by one graph of grouped launches."""

    def __init__(self, masks_list, zbc="periodic"):
        import numpy as np
        self._masks = [np.ascontiguousarray(m, dtype=np.uint8) for m in masks_list]
        self.shapes = [m.shape for m in self._masks]  # (R, H, W)
        descs = [Desc(H, W, R, 1, ZBC[zbc], DENOISER["tv"]) for (R, H, W) in self.shapes]
        self._handle = None
        self._handle = cspnp_batch_create(descs, [m.ctypes.data for m in self._masks], _stream())
        self._ws = None

    def close(self):
        if self._handle is not None:
            cspnp_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self):
        torch = _torch()
        if self._ws is None:
            n = cspnp_batch_workspace_size(self._handle)
            self._ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
        return Plan._ws_ptr(self._ws)

    def allocate(self):
        """Zeroed u, d and empty x per problem."""
        torch = _torch()
        u = [torch.zeros(s, dtype=torch.float32, device="cuda") for s in self.shapes]
        d = [torch.zeros(s, dtype=torch.float32, device="cuda") for s in self.shapes]
        x = [torch.empty(s, dtype=torch.float32, device="cuda") for s in self.shapes]
        return u, d, x

    def solve(self, params_list, y, u, d, x):
        for i, (R, H, W) in enumerate(self.shapes):
            _ptr(y[i], "y[i]", (1, H, W))
            for t, nm in ((u[i], "u[i]"), (d[i], "d[i]"), (x[i], "x[i]")):
                _ptr(t, nm, (R, H, W))
        cspnp_batch_solve(self._handle, params_list, [t.data_ptr() for t in y], [t.data_ptr() for t in u],
                          [t.data_ptr() for t in d], [t.data_ptr() for t in x], self.workspace(), _stream())
        return x, u, d

    def autotune(self, params_list, y, u, d, x):
        cspnp_batch_autotune(self._handle, params_list, [t.data_ptr() for t in y], [t.data_ptr() for t in u],
                             [t.data_ptr() for t in d], [t.data_ptr() for t in x], self.workspace(), _stream())
        return cspnp_batch_get_tv_shape(self._handle)
