"""Small helpers shared by the tests (scene construction for pins)."""
from __future__ import annotations

import numpy as np

from paper_2602_12314_amd import scenes


def gaussians(means, log_scales=None, quats=None, logits=None, queries=None, d=4, seed=0):
    """Explicit Gaussians as float32 arrays (defaults: tiny isotropic, identity rotation)."""
    from oracle.raster import Gaussians
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    rng = np.random.default_rng(seed)
    if log_scales is None:
        log_scales = np.full((n, 3), -3.0)
    if quats is None:
        quats = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    if logits is None:
        logits = np.zeros(n)
    if queries is None:
        queries = rng.standard_normal((n, d))
    queries = np.asarray(queries, np.float64)
    if queries.ndim == 1:
        queries = queries.reshape(n, -1)
    f = lambda a: np.ascontiguousarray(a, np.float32)
    return Gaussians(f(means), f(np.reshape(log_scales, (n, 3))), f(np.reshape(quats, (n, 4))),
                     f(np.reshape(logits, (n,))), f(queries))


def cams_of(*cams):
    return np.stack([c.packed() for c in cams])


def logit(p):
    return float(np.log(p / (1.0 - p)))


def tiny_scene(seed, n=40, w=37, h=29, f=30.0, d=4, pose=scenes.IDENTITY):
    sp = scenes.custom_spec("tiny", n, [scenes.pinhole(w, h, f, pose)], d=d)
    s = scenes.make_scene(sp, seed=seed, with_target=False)
    from oracle.raster import Gaussians
    return Gaussians.of(s), s.cams
