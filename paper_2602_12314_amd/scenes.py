"""Seeded synthetic inputs shaped like the paper's mapping workloads.

This module only draws random numbers and lays out cameras; it holds none of
the method's arithmetic (no projection, compositing, attention or loss), so
both the FP64 oracle tests and the GPU path can consume the same arrays.

Scenes follow the paper's Gaussian parametrisation (Sec. III-A, Eq. 1, plus the
query vector of Sec. III-B): position, orientation quaternion (w, x, y, z),
log-scale, opacity logit and a d-dimensional query.  The paper's datasets
(TUM, Replica, FastCaMo, its own campus capture) are not available; these
seeded scenes stand in for their shapes: Gaussian counts, image sizes,
query / dictionary / feature dimensions and a piecewise-smooth target map.

Camera convention: ``viewmat`` is the 4x4 world->camera transform, row-major,
OpenCV axes (x right, y down, z forward).  Cameras are packed as float32 rows
``[width, height, fx, fy, cx, cy, viewmat[16]]`` (22 floats).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

CAM_FLOATS = 22


@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    viewmat: Tuple[float, ...]  # 16 floats, row-major world->camera

    def packed(self) -> np.ndarray:
        row = [self.width, self.height, self.fx, self.fy, self.cx, self.cy, *self.viewmat]
        return np.asarray(row, dtype=np.float32)

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


IDENTITY = tuple(float(v) for v in np.eye(4).reshape(-1))


def pinhole(width: int, height: int, f: float, pose: Sequence[float] = IDENTITY) -> Camera:
    """Camera with square pixels and the principal point at the image centre."""
    return Camera(width, height, float(np.float32(f)), float(np.float32(f)),
                  float(np.float32(width / 2)), float(np.float32(height / 2)),
                  tuple(float(np.float32(v)) for v in pose))


def look_at_origin(center: Sequence[float]) -> Tuple[float, ...]:
    """World->camera matrix for a level camera at ``center`` looking at the origin.

    World y points down (as in the camera frame), so the camera's y axis is
    world +y and its x axis completes a right-handed frame.
    """
    c = np.asarray(center, dtype=np.float64)
    fwd = -c / np.linalg.norm(c)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd])
    vm = np.eye(4)
    vm[:3, :3] = rot
    vm[:3, 3] = -rot @ c
    return tuple(float(np.float32(v)) for v in vm.reshape(-1))


@dataclass(frozen=True)
class SceneSpec:
    """One workload: scene volume, cameras, and decode sizes."""
    name: str
    n_gauss: int
    boxes: Tuple[Tuple[Tuple[float, float], Tuple[float, float], Tuple[float, float]], ...]
    cams: Tuple[Camera, ...]
    d: int
    M: int
    D: int
    target: str  # "iid" (per-pixel random unit vectors) or "voronoi"
    precision: str = "fp32"
    lambda_tr: float = 0.1
    n_sites: int = 32
    noise: float = 0.05

    @property
    def n_pixels(self) -> int:
        return sum(c.n_pixels for c in self.cams)


def _f(w: int) -> float:
    # Same horizontal field of view as a 640-wide image with f = 525.
    return 525.0 * w / 640.0


def spec(i: int) -> SceneSpec:
    """The five workloads (sizes as stated in the task's configuration list)."""
    if i == 0:
        return SceneSpec("c0_tiny_fp32", 1000, (((-1, 1), (-1, 1), (1, 3)),),
                         (pinhole(80, 60, 70.0),), d=16, M=64, D=512, target="iid")
    if i == 1:
        return SceneSpec("c1_room_640x480", 100_000, (((-4, 4), (-2, 2), (0.5, 8.5)),),
                         (pinhole(640, 480, 525.0),), d=16, M=256, D=512, target="voronoi",
                         precision="bf16")
    if i == 2:
        return SceneSpec("c2_hall_1200x680", 300_000, (((-7.5, 7.5), (-2, 2), (0.5, 15.5)),),
                         (pinhole(1200, 680, _f(1200)),), d=32, M=512, D=768, target="voronoi",
                         precision="bf16")
    if i == 3:
        res = [(320, 240), (480, 360), (640, 480), (640, 480), (640, 480), (960, 540),
               (1200, 680), (1200, 680)]
        cams = []
        for k, (w, h) in enumerate(res):
            th = 2.0 * np.pi * k / 8.0
            cams.append(pinhole(w, h, _f(w), look_at_origin((3 * np.cos(th), 0.0, 3 * np.sin(th)))))
        return SceneSpec("c3_localmap_8views", 500_000, (((-7.5, 7.5), (-2, 2), (-7.5, 7.5)),),
                         tuple(cams), d=16, M=256, D=512, target="voronoi", precision="bf16")
    if i == 4:
        slabs = tuple(((-20, 20), (-5 + 2 * s, -3 + 2 * s), (-20, 20)) for s in range(4))
        return SceneSpec("c4_multifloor_fp8", 2_000_000, slabs,
                         (pinhole(1200, 680, _f(1200)),), d=32, M=1024, D=1024, target="voronoi",
                         precision="fp8")
    raise ValueError(f"unknown workload {i}")


@dataclass
class Scene:
    spec: SceneSpec
    means: np.ndarray          # [N,3] f32
    log_scales: np.ndarray     # [N,3] f32
    quats: np.ndarray          # [N,4] f32 (w,x,y,z), unit norm up to f32 rounding
    opacity_logits: np.ndarray  # [N] f32
    queries: np.ndarray        # [N,d] f32
    K: np.ndarray              # [M,d] f32
    V: np.ndarray              # [M,D] f32
    K0: np.ndarray             # [M,d] f32 (copy of the initial K)
    target: Optional[np.ndarray]  # [n_pix,D] f32, views concatenated in camera order
    cams: np.ndarray           # [n_cams,22] f32

    @property
    def n(self) -> int:
        return self.means.shape[0]


def _target_voronoi(rng: np.random.Generator, spec_: SceneSpec) -> np.ndarray:
    D = spec_.D
    protos = rng.standard_normal((spec_.n_sites, D))
    protos /= np.linalg.norm(protos, axis=1, keepdims=True)
    out = np.empty((spec_.n_pixels, D), dtype=np.float32)
    off = 0
    for cam in spec_.cams:
        sites = rng.uniform(0.0, 1.0, size=(spec_.n_sites, 2)) * np.array([cam.width, cam.height])
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        pix = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float64)
        # nearest site per pixel, chunked to bound memory
        lab = np.empty(pix.shape[0], dtype=np.int64)
        for s in range(0, pix.shape[0], 1 << 16):
            dd = ((pix[s:s + (1 << 16), None, :] - sites[None]) ** 2).sum(-1)
            lab[s:s + (1 << 16)] = dd.argmin(1)
        for s in range(0, pix.shape[0], 1 << 15):
            e = min(pix.shape[0], s + (1 << 15))
            t = protos[lab[s:e]] + spec_.noise * rng.standard_normal((e - s, D))
            t /= np.linalg.norm(t, axis=1, keepdims=True)
            out[off + s:off + e] = t
        off += pix.shape[0]
    return out


def _target_iid(rng: np.random.Generator, spec_: SceneSpec) -> np.ndarray:
    t = rng.standard_normal((spec_.n_pixels, spec_.D))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return t.astype(np.float32)


def make_scene(spec_: SceneSpec, seed: int = 0, with_target: bool = True) -> Scene:
    """Draw a scene.  Draw order is fixed: means, log-scales, quaternions,
    opacity logits, queries, K, V, then the target (prototypes, sites, noise)."""
    rng = np.random.default_rng(seed)
    N = spec_.n_gauss
    nb = len(spec_.boxes)
    per = [N // nb + (1 if b < N % nb else 0) for b in range(nb)]
    parts = []
    for b, box in enumerate(spec_.boxes):
        lo = np.array([box[0][0], box[1][0], box[2][0]], dtype=np.float64)
        hi = np.array([box[0][1], box[1][1], box[2][1]], dtype=np.float64)
        parts.append(lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(per[b], 3)))
    means = np.concatenate(parts, axis=0)
    log_scales = rng.normal(-3.0, 0.3, size=(N, 3))
    q = rng.standard_normal((N, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.standard_normal(N)
    queries = rng.standard_normal((N, spec_.d))
    K = rng.standard_normal((spec_.M, spec_.d))
    V = rng.standard_normal((spec_.M, spec_.D))
    target = None
    if with_target:
        target = _target_iid(rng, spec_) if spec_.target == "iid" else _target_voronoi(rng, spec_)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(spec_, f32(means), f32(log_scales), f32(q), f32(logits), f32(queries),
                 f32(K), f32(V), f32(K).copy(), target,
                 np.stack([c.packed() for c in spec_.cams]))


def custom_spec(name: str, n_gauss: int, cams: Sequence[Camera], d: int = 16, M: int = 64,
                D: int = 128, box=((-1, 1), (-1, 1), (1, 3)), target: str = "iid") -> SceneSpec:
    """A small workload for tests (ragged images, few Gaussians, odd sizes)."""
    return SceneSpec(name, n_gauss, (box,), tuple(cams), d=d, M=M, D=D, target=target)


def pixel_offsets(cams: np.ndarray) -> np.ndarray:
    """Start of each view in the concatenated pixel order."""
    n = (cams[:, 0].astype(np.int64) * cams[:, 1].astype(np.int64))
    return np.concatenate([[0], np.cumsum(n)])
