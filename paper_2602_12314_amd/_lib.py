"""ctypes binding of ``liblatentam.so`` -- argument marshalling only.

Every function here forwards to the C ABI of include/latentam.h with the same
name minus the ``lam_`` prefix.  Tensors are passed as device pointers
(``data_ptr()``); the stream is torch's current HIP stream unless given; the
library context is ``ctx`` (a ``Context``) or the current device's default
one.  There is no fallback: if the library is not built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblatentam.so")

LAM_OK, LAM_ERR_INVALID_ARG, LAM_ERR_UNSUPPORTED, LAM_ERR_CAPACITY, LAM_ERR_HIP = 0, -1, -2, -3, -4
LAM_FP32, LAM_BF16, LAM_FP8_E4M3 = 0, 1, 2
PRECISIONS = {"fp32": LAM_FP32, "bf16": LAM_BF16, "fp8": LAM_FP8_E4M3}
CAM_FLOATS = 22

_lib = None


class TiedParams(C.Structure):
    """lam_tied_params: temperature and loss weights of the tied decode."""
    _fields_ = [("tau", C.c_float), ("lambda_cos", C.c_float), ("lambda_2", C.c_float),
                ("lambda_D", C.c_float), ("delta", C.c_float)]


class LamError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2602_12314_amd.build` "
                               "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64, f32 = C.c_void_p, C.c_int, C.c_uint64, C.c_float
        pu64, pi32 = C.POINTER(C.c_uint64), C.POINTER(C.c_int)
        sig = {
            "lam_status_string": (C.c_char_p, [i32]),
            "lam_version": (i32, []),
            "lam_create": (i32, [i32, C.c_char_p, C.POINTER(vp)]),
            "lam_destroy": (None, [vp]),
            "lam_ctx_configure": (i32, [vp, C.c_char_p]),
            "lam_ctx_get": (i32, [vp, C.c_char_p, pi32]),
            "lam_profile_enable": (i32, [vp, i32]),
            "lam_profile_read": (i32, [vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
            "lam_render_workspace_size": (i32, [vp, i32, i32, vp, i32, i32, i32, u64, pu64]),
            "lam_render_forward": (i32, [vp, vp, vp, vp, vp, vp, i32, i32, vp, i32, i32, i32, vp, vp, vp,
                                         u64, u64, vp]),
            "lam_render_backward": (i32, [vp, vp, vp, vp, vp, vp, i32, i32, vp, i32, i32, i32, vp, vp, vp,
                                          vp, vp, vp, vp, u64, u64, vp]),
            "lam_render_counters": (i32, [vp, vp, vp, pu64, pi32]),
            "lam_render_debug_views": (i32, [vp, vp, i32, i32, vp, i32, i32, i32, u64] + [C.POINTER(vp)] * 6),
            "lam_decode_workspace_size": (i32, [vp, i32, i32, i32, i32, i32, pu64]),
            "lam_decode_loss": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp, f32, vp, vp, vp, vp,
                                      vp, vp, u64, vp]),
            "lam_decode_loss_overlap": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp, f32, vp, vp, vp, vp,
                                              vp, vp, u64, vp, vp]),
            "lam_decode_forward": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp, u64, vp]),
            "lam_decode_forward_noalloc": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp]),
            "lam_decode_backward": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, u64,
                                          vp]),
            "lam_decode_tied_workspace_size": (i32, [vp, i32, i32, i32, i32, i32, pu64]),
            "lam_decode_tied_loss": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp, C.POINTER(TiedParams),
                                           vp, vp, vp, vp, vp, u64, vp]),
            "lam_render_rgbd_forward": (i32, [vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, i32, i32, i32, vp, vp, vp,
                                              vp, vp, u64, u64, vp]),
            "lam_render_rgbd_backward": (i32, [vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, i32, i32, i32, vp, vp, vp,
                                               vp, vp, vp, vp, vp, vp, vp, u64, u64, vp]),
            "lam_rgbd_l1_workspace_size": (i32, [vp, i32, pu64]),
            "lam_ssim_workspace_size": (i32, [vp, vp, i32, pu64]),
            "lam_ssim_loss": (i32, [vp, vp, vp, vp, i32, f32, vp, vp, i32, vp, u64, vp]),
            "lam_rgbd_l1_loss": (i32, [vp, vp, vp, vp, vp, i32, f32, f32, vp, vp, vp, vp, u64, vp]),
            "lam_kmeans_workspace_size": (i32, [vp, i32, i32, i32, i32, pu64]),
            "lam_kmeans_assign": (i32, [vp, i32, vp, i32, i32, vp, i32, vp, vp, vp, u64, vp]),
            "lam_kmeans_lloyd": (i32, [vp, i32, vp, vp, i32, i32, vp, i32, i32, vp, vp, vp, vp, u64, vp]),
            "lam_stream_kmeans_workspace_size": (i32, [vp, i32, i32, i32, i32, i32, i32, pu64]),
            "lam_stream_kmeans": (i32, [vp, i32, vp, i32, i32, vp, vp, i32, i32, vp, i32, i32, i32, vp, vp, vp,
                                        u64, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().lam_status_string(int(status)).decode()


def check(status: int, where: str):
    if status != LAM_OK:
        raise LamError(status, where)


def _p(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _cams(cams) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(cams, dtype=np.float32).reshape(-1, CAM_FLOATS))
    return a


# ------------------------------------------------------------------ render

SCHEDULES = {"per_tile": 0, "persistent": 1, "auto": 2}


def render_workspace_size(n_gauss, d, cams, tile_w, tile_h, capacity, ctx=None) -> int:
    cams = _cams(cams)
    out = C.c_uint64()
    check(lib().lam_render_workspace_size(_size_ctx(ctx), n_gauss, d, cams.ctypes.data_as(C.c_void_p), cams.shape[0],
                                          tile_w, tile_h, capacity, C.byref(out)),
          "lam_render_workspace_size")
    return int(out.value)


def render_forward(g, cams, tile_w, tile_h, Q, T_final, ws, capacity, stream=None, ctx=None):
    cams = _cams(cams)
    check(lib().lam_render_forward(_ctx(ctx), _p(g.means), _p(g.log_scales), _p(g.quats), _p(g.opacity_logits),
                                   _p(g.queries), g.means.shape[0], g.queries.shape[1],
                                   cams.ctypes.data_as(C.c_void_p), cams.shape[0], tile_w, tile_h,
                                   _p(Q), _p(T_final), _p(ws), ws.numel() * ws.element_size(),
                                   capacity, _stream(stream)), "lam_render_forward")


def render_backward(g, cams, tile_w, tile_h, dQ, grads, ws, capacity, stream=None, ctx=None):
    cams = _cams(cams)
    check(lib().lam_render_backward(_ctx(ctx), _p(g.means), _p(g.log_scales), _p(g.quats), _p(g.opacity_logits),
                                    _p(g.queries), g.means.shape[0], g.queries.shape[1],
                                    cams.ctypes.data_as(C.c_void_p), cams.shape[0], tile_w, tile_h,
                                    _p(dQ), _p(grads.means), _p(grads.log_scales), _p(grads.quats),
                                    _p(grads.opacity_logits), _p(grads.queries), _p(ws),
                                    ws.numel() * ws.element_size(), capacity, _stream(stream)),
          "lam_render_backward")


def render_rgbd_forward(g, colors, cams, tile_w, tile_h, Q, rgb, depth, T_final, ws, capacity, stream=None, ctx=None):
    cams = _cams(cams)
    check(lib().lam_render_rgbd_forward(_ctx(ctx), _p(g.means), _p(g.log_scales), _p(g.quats), _p(g.opacity_logits),
                                        _p(g.queries), _p(colors), g.means.shape[0], g.queries.shape[1],
                                        cams.ctypes.data_as(C.c_void_p), cams.shape[0], tile_w, tile_h,
                                        _p(Q), _p(rgb), _p(depth), _p(T_final), _p(ws),
                                        ws.numel() * ws.element_size(), capacity, _stream(stream)),
          "lam_render_rgbd_forward")


def render_rgbd_backward(g, colors, cams, tile_w, tile_h, dQ, d_rgb, d_depth, grads, d_colors, ws, capacity,
                         stream=None, ctx=None):
    cams = _cams(cams)
    check(lib().lam_render_rgbd_backward(_ctx(ctx), _p(g.means), _p(g.log_scales), _p(g.quats), _p(g.opacity_logits),
                                         _p(g.queries), _p(colors), g.means.shape[0], g.queries.shape[1],
                                         cams.ctypes.data_as(C.c_void_p), cams.shape[0], tile_w, tile_h,
                                         _p(dQ), _p(d_rgb), _p(d_depth), _p(grads.means),
                                         _p(grads.log_scales), _p(grads.quats), _p(grads.opacity_logits),
                                         _p(grads.queries), _p(d_colors), _p(ws),
                                         ws.numel() * ws.element_size(), capacity, _stream(stream)),
          "lam_render_rgbd_backward")


def rgbd_l1_workspace_size(n, ctx=None) -> int:
    out = C.c_uint64()
    check(lib().lam_rgbd_l1_workspace_size(_size_ctx(ctx), int(n), C.byref(out)), "lam_rgbd_l1_workspace_size")
    return int(out.value)


def rgbd_l1_loss(rgb, rgb_obs, depth, depth_obs, lambda_rgb, lambda_depth, loss, d_rgb, d_depth, ws,
                 stream=None, ctx=None):
    check(lib().lam_rgbd_l1_loss(_ctx(ctx), _p(rgb), _p(rgb_obs), _p(depth), _p(depth_obs), depth.shape[0],
                                 float(lambda_rgb), float(lambda_depth), _p(loss), _p(d_rgb), _p(d_depth),
                                 _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
          "lam_rgbd_l1_loss")


def ssim_workspace_size(cams, ctx=None) -> int:
    cams = _cams(cams)
    out = C.c_uint64()
    check(lib().lam_ssim_workspace_size(_size_ctx(ctx), cams.ctypes.data_as(C.c_void_p), cams.shape[0], C.byref(out)),
          "lam_ssim_workspace_size")
    return int(out.value)


def ssim_loss(rgb, rgb_obs, cams, lam, loss, d_rgb, accumulate, ws, stream=None, ctx=None):
    cams = _cams(cams)
    check(lib().lam_ssim_loss(_ctx(ctx), _p(rgb), _p(rgb_obs), cams.ctypes.data_as(C.c_void_p), cams.shape[0], float(lam),
                              _p(loss), _p(d_rgb), 1 if accumulate else 0, _p(ws), ws.numel() * ws.element_size(),
                              _stream(stream)), "lam_ssim_loss")


def render_counters(ws, stream=None, ctx=None):
    """BLOCKING: (pairs needed, overflowed) of the last forward on ``ws``."""
    need, over = C.c_uint64(), C.c_int()
    st = lib().lam_render_counters(_ctx(ctx), _p(ws), _stream(stream), C.byref(need), C.byref(over))
    if st not in (LAM_OK, LAM_ERR_CAPACITY):
        check(st, "lam_render_counters")
    return int(need.value), bool(over.value)


def render_debug_views(ws, n_gauss, d, cams, tile_w, tile_h, capacity, ctx=None):
    cams = _cams(cams)
    ptrs = [C.c_void_p() for _ in range(6)]
    check(lib().lam_render_debug_views(_size_ctx(ctx), _p(ws), n_gauss, d, cams.ctypes.data_as(C.c_void_p),
                                       cams.shape[0], tile_w, tile_h, capacity,
                                       *[C.byref(p) for p in ptrs]), "lam_render_debug_views")
    return [p.value for p in ptrs]


# ------------------------------------------------------------------ decode

DECODE_SHAPES = {"px32": 0, "px64": 1}


def decode_workspace_size(precision, n, d, M, D, ctx=None) -> int:
    out = C.c_uint64()
    check(lib().lam_decode_workspace_size(_size_ctx(ctx), PRECISIONS.get(precision, precision), n, d, M, D,
                                          C.byref(out)), "lam_decode_workspace_size")
    return int(out.value)


def decode_loss(precision, Q, K, V, target, K0, lambda_tr, loss, dQ, dK, dV, row_cos, ws, stream=None, ctx=None):
    n, d = Q.shape
    M, D = V.shape
    check(lib().lam_decode_loss(_ctx(ctx), PRECISIONS.get(precision, precision), _p(Q), n, d, _p(K), _p(V), M, D,
                                _p(target), _p(K0), float(lambda_tr), _p(loss), _p(dQ), _p(dK), _p(dV),
                                _p(row_cos), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
          "lam_decode_loss")


def decode_loss_overlap(precision, Q, K, V, target, K0, lambda_tr, loss, dQ, dK, dV, row_cos, ws, dict_stream,
                        stream=None, ctx=None):
    n, d = Q.shape
    M, D = V.shape
    check(lib().lam_decode_loss_overlap(_ctx(ctx), PRECISIONS.get(precision, precision), _p(Q), n, d, _p(K), _p(V), M, D,
                                        _p(target), _p(K0), float(lambda_tr), _p(loss), _p(dQ), _p(dK), _p(dV),
                                        _p(row_cos), _p(ws), ws.numel() * ws.element_size(), _stream(stream),
                                        _stream(dict_stream)),
          "lam_decode_loss_overlap")


def decode_forward(precision, Q, K, V, F, ws, stream=None, ctx=None):
    n, d = Q.shape
    M, D = V.shape
    check(lib().lam_decode_forward(_ctx(ctx), PRECISIONS.get(precision, precision), _p(Q), n, d, _p(K), _p(V), M, D,
                                   _p(F), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
          "lam_decode_forward")


NOALLOC_SCRATCH_BYTES = 8 << 20  # LAM_NOALLOC_SCRATCH_BYTES


def decode_forward_noalloc(precision, Q, K, V, F, stream=None, ctx=None):
    """lam_decode_forward without a workspace: the dictionary is prepared in
    the library's static per-GPU scratch (calls on one GPU must not overlap)."""
    n, d = Q.shape
    M, D = V.shape
    check(lib().lam_decode_forward_noalloc(_ctx(ctx), PRECISIONS.get(precision, precision), _p(Q), n, d, _p(K),
                                           _p(V), M, D, _p(F), _stream(stream)),
          "lam_decode_forward_noalloc")


def decode_backward(precision, Q, K, V, dF, dQ, dK, dV, ws, stream=None, ctx=None):
    n, d = Q.shape
    M, D = V.shape
    check(lib().lam_decode_backward(_ctx(ctx), PRECISIONS.get(precision, precision), _p(Q), n, d, _p(K), _p(V), M,
                                    D, _p(dF), _p(dQ), _p(dK), _p(dV), _p(ws),
                                    ws.numel() * ws.element_size(), _stream(stream)),
          "lam_decode_backward")


def decode_tied_workspace_size(precision, n, ds, M, df, ctx=None) -> int:
    out = C.c_uint64()
    check(lib().lam_decode_tied_workspace_size(_size_ctx(ctx), PRECISIONS.get(precision, precision), n, ds, M, df,
                                               C.byref(out)), "lam_decode_tied_workspace_size")
    return int(out.value)


def decode_tied_loss(precision, Q, W, D, target, D0, params, loss, dQ, dW, dD, ws, stream=None, ctx=None):
    n, ds = Q.shape
    M, df = D.shape
    p = TiedParams(*[float(params[k]) for k in ("tau", "lambda_cos", "lambda_2", "lambda_D", "delta")])
    check(lib().lam_decode_tied_loss(_ctx(ctx), PRECISIONS.get(precision, precision), _p(Q), n, ds, _p(W), _p(D), M, df,
                                     _p(target), _p(D0), C.byref(p), _p(loss), _p(dQ), _p(dW), _p(dD), _p(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)),
          "lam_decode_tied_loss")


# ------------------------------------------------------------ streaming K-means

KMEANS_PRECISIONS = ("fp32", "bf16")


def kmeans_workspace_size(precision, n, D, k, ctx=None) -> int:
    out = C.c_uint64()
    check(lib().lam_kmeans_workspace_size(_size_ctx(ctx), PRECISIONS.get(precision, precision), n, D, k, C.byref(out)),
          "lam_kmeans_workspace_size")
    return int(out.value)


def kmeans_assign(precision, X, C_, assign, d2, ws, stream=None, ctx=None):
    n, D = X.shape
    check(lib().lam_kmeans_assign(_ctx(ctx), PRECISIONS.get(precision, precision), _p(X), n, D, _p(C_), C_.shape[0],
                                  _p(assign), _p(d2), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
          "lam_kmeans_assign")


def kmeans_lloyd(precision, X, weights, C0, iters, C_out, W, assign, ws, stream=None, ctx=None):
    n, D = X.shape
    check(lib().lam_kmeans_lloyd(_ctx(ctx), PRECISIONS.get(precision, precision), _p(X), _p(weights), n, D, _p(C0),
                                 C0.shape[0], int(iters), _p(C_out), _p(W), _p(assign), _p(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)),
          "lam_kmeans_lloyd")


def stream_kmeans_workspace_size(precision, n, D, Kp, K, m, ctx=None) -> int:
    out = C.c_uint64()
    check(lib().lam_stream_kmeans_workspace_size(_size_ctx(ctx), PRECISIONS.get(precision, precision), n, D, Kp, K, m,
                                                 C.byref(out)), "lam_stream_kmeans_workspace_size")
    return int(out.value)


def stream_kmeans(precision, F, D_prev, w_prev, K, seeds, iters_local, iters_global, D_out, W_out, ws,
                  stream=None, ctx=None):
    """seeds: host int32 array (numpy), read before the call returns."""
    n, D = F.shape
    Kp = 0 if D_prev is None else D_prev.shape[0]
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.int32).reshape(-1))
    check(lib().lam_stream_kmeans(_ctx(ctx), PRECISIONS.get(precision, precision), _p(F), n, D, _p(D_prev), _p(w_prev), Kp,
                                  int(K), sd.ctypes.data_as(C.c_void_p), sd.shape[0], int(iters_local),
                                  int(iters_global), _p(D_out), _p(W_out), _p(ws), ws.numel() * ws.element_size(),
                                  _stream(stream)),
          "lam_stream_kmeans")


# ------------------------------------------------------------------ context

class Context:
    """A ``lam_ctx``: the device it was made for and its launch options
    (``raster_schedule``, ``decode_shape``, ``decode_splits``; see
    include/latentam.h).  Destroyed with the object."""

    def __init__(self, device=None, options=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        ptr = C.c_void_p()
        js = None if options is None else json.dumps(_encode_options(options)).encode()
        check(lib().lam_create(self.device, js, C.byref(ptr)), "lam_create")
        self._ptr = ptr
        self._destroy = lib().lam_destroy

    @property
    def ptr(self):
        return self._ptr

    def configure(self, **options):
        check(lib().lam_ctx_configure(self._ptr, json.dumps(_encode_options(options)).encode()),
              "lam_ctx_configure")

    def get(self, key: str) -> int:
        v = C.c_int()
        check(lib().lam_ctx_get(self._ptr, key.encode(), C.byref(v)), "lam_ctx_get")
        return int(v.value)

    def options(self) -> dict:
        return {k: self.get(k) for k in ("raster_schedule", "decode_shape", "decode_splits")}

    def profile_enable(self, on: bool):
        check(lib().lam_profile_enable(self._ptr, 1 if on else 0), "lam_profile_enable")

    def profile_read(self, name: str):
        """BLOCKING: (total ms, launches) of kernel ``name`` since the last read."""
        tot, cnt = C.c_double(), C.c_int()
        check(lib().lam_profile_read(self._ptr, name.encode(), C.byref(tot), C.byref(cnt)), "lam_profile_read")
        return float(tot.value), int(cnt.value)

    def close(self):
        if getattr(self, "_ptr", None) is not None and self._ptr.value:
            self._destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _encode_options(options: dict) -> dict:
    out = {}
    for k, v in options.items():
        if k == "raster_schedule":
            v = SCHEDULES.get(v, v)
        elif k == "decode_shape":
            v = DECODE_SHAPES.get(v, v)
        out[k] = int(v)
    return out


_defaults = {}


def default_context(device=None) -> Context:
    """The context a call uses when none is given: one per device, made on
    first use with the default options."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    c = _defaults.get(dev)
    if c is None:
        c = _defaults[dev] = Context(dev)
    return c


def _ctx(ctx):
    return (ctx if ctx is not None else default_context()).ptr


def _size_ctx(ctx):
    """Context for a host-only size query: the given one, else the current
    device's default context if it exists, else NULL (the default options)."""
    if ctx is not None:
        return ctx.ptr
    if _defaults:
        import torch
        c = _defaults.get(torch.cuda.current_device())
        if c is not None:
            return c.ptr
    return None
