"""ctypes front end of the C oracle for the query-map renderer.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU-baseline leg).
See raster_oracle.c for what is computed and which passages it follows.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_build.ensure_built())
        vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
        _lib.orc_project.restype = i64
        _lib.orc_project.argtypes = [i32, vp, vp, vp, vp, i32, vp] + [vp] * 8
        _lib.orc_project_decisions64.restype = i64
        _lib.orc_project_decisions64.argtypes = [i32, vp, vp, vp, vp, i32, vp] + [vp] * 5
        _lib.orc_exp_cw.restype = None
        _lib.orc_exp_cw.argtypes = [i64, vp, vp]
        _lib.orc_bin.restype = i64
        _lib.orc_bin.argtypes = [i32, vp, vp, vp, vp, i32, vp, i32, i32, i64, vp, vp, vp, vp]
        _lib.orc_num_tiles.restype = i64
        _lib.orc_num_tiles.argtypes = [i32, vp, i32, i32]
        _lib.orc_render_forward.restype = i32
        _lib.orc_render_forward.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, vp, i32, i32] + [vp] * 8
        _lib.orc_render_bruteforce.restype = i32
        _lib.orc_render_bruteforce.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        _lib.orc_render_backward.restype = i32
        _lib.orc_render_backward.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, vp, i32, i32, vp] + [vp] * 7
        _lib.orc_num_threads.restype = i32
        _lib.orc_set_num_threads.restype = None
        _lib.orc_set_num_threads.argtypes = [i32]
        _lib.orc_render_window.restype = i32
        _lib.orc_render_window.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp]
        _lib.orc_fd_window.restype = i32
        _lib.orc_fd_window.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, i32, vp, vp,
                                       C.c_double, vp, vp]
        _lib.orc_pixel_walks.restype = i32
        _lib.orc_pixel_walks.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, vp, i32, i32, i32, vp, i32, vp, vp,
                                         vp, vp, vp]
    return _lib


def _c(a, dt=np.float32):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass
class Gaussians:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    queries: np.ndarray

    @classmethod
    def of(cls, scene) -> "Gaussians":
        return cls(_c(scene.means), _c(scene.log_scales), _c(scene.quats),
                   _c(scene.opacity_logits), _c(scene.queries))

    @property
    def n(self) -> int:
        return self.means.shape[0]

    @property
    def d(self) -> int:
        return self.queries.shape[1]

    def geom_args(self):
        return [_ptr(self.means), _ptr(self.log_scales), _ptr(self.quats), _ptr(self.opacity_logits)]


def n_pixels(cams: np.ndarray) -> int:
    return int((cams[:, 0].astype(np.int64) * cams[:, 1].astype(np.int64)).sum())


def num_tiles(cams, tw=16, th=16) -> int:
    cams = _c(cams)
    return int(lib().orc_num_tiles(cams.shape[0], _ptr(cams), tw, th))


def project(g: Gaussians, cams):
    cams = _c(cams)
    R = cams.shape[0] * g.n
    out = dict(uv=np.zeros((R, 2)), conic=np.zeros((R, 3)), opacity=np.zeros(R),
               radius=np.zeros(R), rect=np.zeros((R, 4), np.int32),
               depth_key=np.zeros(R, np.uint32), vis=np.zeros(R, np.uint8), z=np.zeros(R))
    nv = lib().orc_project(g.n, *g.geom_args(), cams.shape[0], _ptr(cams), _ptr(out["uv"]),
                           _ptr(out["conic"]), _ptr(out["opacity"]), _ptr(out["radius"]),
                           _ptr(out["rect"]), _ptr(out["depth_key"]), _ptr(out["vis"]),
                           _ptr(out["z"]))
    out["n_visible"] = int(nv)
    return out


def project_decisions64(g: Gaussians, cams):
    """The projection's integer decisions taken in FP64, their margin (pixels,
    or depth units for the near plane) and the float32 screen mean."""
    cams = _c(cams)
    R = cams.shape[0] * g.n
    out = dict(rect=np.zeros((R, 4), np.int32), depth_key=np.zeros(R, np.uint32), vis=np.zeros(R, np.uint8),
               margin=np.zeros(R), uv32=np.zeros((R, 2), np.float32))
    lib().orc_project_decisions64(g.n, *g.geom_args(), cams.shape[0], _ptr(cams), _ptr(out["rect"]),
                                  _ptr(out["depth_key"]), _ptr(out["vis"]), _ptr(out["margin"]),
                                  _ptr(out["uv32"]))
    return out


def exp_cw(x):
    """The float32 exp of the projection (Cody-Waite reduction, Taylor polynomial)."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().orc_exp_cw(x.size, _ptr(x), _ptr(y))
    return y


def bin_sort(g: Gaussians, cams, tw=16, th=16):
    """Tile instances sorted by (tile, depth key, record) and per-tile ranges."""
    cams = _c(cams)
    cnt = lib().orc_bin(g.n, *g.geom_args(), cams.shape[0], _ptr(cams), tw, th, 0,
                        None, None, None, None)
    tiles = np.zeros(max(cnt, 1), np.uint32)
    depths = np.zeros(max(cnt, 1), np.uint32)
    recs = np.zeros(max(cnt, 1), np.uint32)
    ranges = np.zeros((num_tiles(cams, tw, th), 2), np.uint32)
    lib().orc_bin(g.n, *g.geom_args(), cams.shape[0], _ptr(cams), tw, th, cnt, _ptr(tiles),
                  _ptr(depths), _ptr(recs), _ptr(ranges))
    return dict(count=int(cnt), tiles=tiles[:cnt], depths=depths[:cnt], recs=recs[:cnt],
                ranges=ranges)


def render_forward(g: Gaussians, cams, tw=16, th=16):
    """Query map Q (Eq. 4), depth map Z (the same blend of the centres'
    camera-space depths), final transmittance and per-pixel bookkeeping."""
    cams = _c(cams)
    P = n_pixels(cams)
    out = dict(Q=np.zeros((P, g.d)), T_final=np.zeros(P), n_contrib=np.zeros(P, np.int32),
               n_blended=np.zeros(P, np.int32), n_pairs=np.zeros(P, np.int32),
               margin=np.zeros(P), hash=np.zeros(P, np.uint64), Z=np.zeros(P))
    lib().orc_render_forward(g.n, g.d, *g.geom_args(), _ptr(g.queries), cams.shape[0],
                             _ptr(cams), tw, th, _ptr(out["Q"]), _ptr(out["T_final"]),
                             _ptr(out["n_contrib"]), _ptr(out["n_blended"]),
                             _ptr(out["n_pairs"]), _ptr(out["margin"]), _ptr(out["hash"]),
                             _ptr(out["Z"]))
    return out


def render_bruteforce(g: Gaussians, cams):
    cams = _c(cams)
    P = n_pixels(cams)
    out = dict(Q=np.zeros((P, g.d)), T_final=np.zeros(P), n_blended=np.zeros(P, np.int32),
               Z=np.zeros(P))
    lib().orc_render_bruteforce(g.n, g.d, *g.geom_args(), _ptr(g.queries), cams.shape[0],
                                _ptr(cams), _ptr(out["Q"]), _ptr(out["T_final"]),
                                _ptr(out["n_blended"]), _ptr(out["Z"]))
    return out


def render_backward(g: Gaussians, cams, dQ, tw=16, th=16, with_rec: bool = False, dZ=None):
    """Adjoint for the upstream gradients dQ [P, d] and (optional) dZ [P]."""
    cams = _c(cams)
    dQ = _c(dQ, np.float64)
    dZ = None if dZ is None else _c(dZ, np.float64)
    n, d = g.n, g.d
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), queries=np.zeros((n, d)))
    rec = np.zeros((cams.shape[0] * n, 6)) if with_rec else None
    lib().orc_render_backward(n, d, *g.geom_args(), _ptr(g.queries), cams.shape[0], _ptr(cams),
                              tw, th, _ptr(dQ), _ptr(out["means"]), _ptr(out["log_scales"]),
                              _ptr(out["quats"]), _ptr(out["opacity_logits"]),
                              _ptr(out["queries"]), _ptr(rec), _ptr(dZ))
    if with_rec:
        out["rec"] = rec
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int):
    """Threads of the oracle's OpenMP regions from now on."""
    lib().orc_set_num_threads(int(n))


# parameter index of a probe in fd_window: 0-2 mean, 3-5 log-scale, 6-9 quaternion,
# 10 opacity logit, 11.. query
PARAM_SLICES = {"means": (0, 3), "log_scales": (3, 6), "quats": (6, 10), "opacity_logits": (10, 11)}


def render_window(g: Gaussians, cam, x0, y0, ww, wh):
    """Q [ww*wh, d], T_final and decision signatures of a pixel window of one
    camera (row-major inside the window), by the tile-free definition."""
    cam = _c(np.asarray(cam).reshape(-1)[:22])
    out = dict(Q=np.zeros((ww * wh, g.d)), T_final=np.zeros(ww * wh), hash=np.zeros(ww * wh, np.uint64))
    lib().orc_render_window(g.n, g.d, *g.geom_args(), _ptr(g.queries), _ptr(cam), x0, y0, ww, wh,
                            _ptr(out["Q"]), _ptr(out["T_final"]), _ptr(out["hash"]))
    return out


def fd_window(g: Gaussians, cam, x0, y0, ww, wh, w, probe_gauss, probe_param, hrel=1e-5):
    """Central differences of sum_p w_p . Q_p over the window for each probe
    (Gaussian, parameter index); returns (fd, ok) where ok marks probes whose
    stencil changes no pixel's decisions."""
    cam = _c(np.asarray(cam).reshape(-1)[:22])
    w = _c(w, np.float64).reshape(ww * wh, g.d)
    pg = _c(probe_gauss, np.int32)
    pk = _c(probe_param, np.int32)
    fd = np.zeros(len(pg))
    ok = np.zeros(len(pg), np.int32)
    lib().orc_fd_window(g.n, g.d, *g.geom_args(), _ptr(g.queries), _ptr(cam), x0, y0, ww, wh, _ptr(w), len(pg),
                        _ptr(pg), _ptr(pk), float(hrel), _ptr(fd), _ptr(ok))
    return fd, ok.astype(bool)


def pixel_walks(g: Gaussians, cams, pixels, max_len=4096, tw=16, th=16):
    """Per listed pixel: blended record ids, their alphas and the transmittance
    before each (arrays [npix, max_len], valid up to count), count, T_final."""
    cams = _c(cams)
    px = _c(pixels, np.int64)
    k = len(px)
    out = dict(recs=np.full((k, max_len), -1, np.int64), alpha=np.zeros((k, max_len)),
               T_before=np.zeros((k, max_len)), count=np.zeros(k, np.int32), T_final=np.zeros(k))
    lib().orc_pixel_walks(g.n, g.d, *g.geom_args(), _ptr(g.queries), cams.shape[0], _ptr(cams), tw, th, k,
                          _ptr(px), max_len, _ptr(out["recs"]), _ptr(out["alpha"]), _ptr(out["T_before"]),
                          _ptr(out["count"]), _ptr(out["T_final"]))
    return out
