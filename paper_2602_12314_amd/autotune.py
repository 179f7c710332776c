"""Autotuner for the render tile shape and the decode block shape.

The rendered query map does not depend on the tile shape (each Gaussian is
blended into exactly the pixels of its footprint), so the shape is a pure
performance choice: ``best_tile`` times render forward + backward for each
candidate on the caller's own scene and cameras and keeps the fastest.
``best_decode_shape`` times the decode + loss + gradients call for its two
workgroup shapes (32 pixels x 4 waves, 64 pixels x 8 waves) on inputs of the
caller's sizes; the results agree to rounding.  Results are cached in JSON
keyed by GPU architecture and workload shape (``$LAM_AUTOTUNE_CACHE``, default
``~/.cache/latentam/autotune.json``).
"""
from __future__ import annotations

import json
import os
import time
from typing import Iterable, Optional, Tuple

import numpy as np
import torch

from . import _lib, ops

CANDIDATES = ((16, 16), (8, 8), (16, 8), (8, 16), (32, 8), (8, 32), (16, 4), (32, 4))


def cache_path() -> str:
    return os.environ.get("LAM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "latentam", "autotune.json"))


def _key(cams: np.ndarray, n_gauss: int, d: int) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    views = ",".join(f"{int(c[0])}x{int(c[1])}" for c in cams)
    return f"{arch}|N={n_gauss}|d={d}|views={views}"


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_tile(g: ops.Gaussians, cams, tile, reps: int = 5, warmup: int = 2) -> float:
    """Median ms of render forward + backward with a random upstream gradient."""
    r = ops.Renderer(cams, g.n, g.d, tile=tile)
    Q, T = r.forward(g)
    dQ = torch.randn_like(Q)
    out = g.zeros_like()
    for _ in range(warmup):
        r.forward(g, Q, T, check=False)
        r.backward(g, dQ, out=out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r.forward(g, Q, T, check=False)
        r.backward(g, dQ, out=out)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    assert not r.counters()[1]
    return float(np.median(ts))


def best_tile(g: ops.Gaussians, cams, candidates: Iterable[Tuple[int, int]] = CANDIDATES,
              use_cache: bool = True, reps: int = 5) -> Tuple[Tuple[int, int], dict]:
    cams = np.asarray(cams, np.float32).reshape(-1, 22)
    key = _key(cams, g.n, g.d)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        ent = db[key]
        return tuple(ent["tile"]), ent["ms"]
    times = {f"{tw}x{th}": time_tile(g, cams, (tw, th), reps=reps) for tw, th in candidates}
    best = min(times, key=times.get)
    tile = tuple(int(v) for v in best.split("x"))
    if use_cache:
        db[key] = {"tile": list(tile), "ms": times}
        _store(db)
    return tile, times


def time_decode_shape(precision: str, n: int, d: int, M: int, D: int, shape: str, reps: int = 5,
                      warmup: int = 2) -> float:
    """Median ms of decode + loss + gradients with the given block shape."""
    dev = torch.device("cuda", torch.cuda.current_device())
    gen = torch.Generator(device=dev).manual_seed(0)
    Q = torch.randn((n, d), device=dev, generator=gen)
    K = torch.randn((M, d), device=dev, generator=gen)
    V = torch.randn((M, D), device=dev, generator=gen)
    T = torch.nn.functional.normalize(torch.randn((n, D), device=dev, generator=gen), dim=1)
    dec = ops.Decoder(precision, n, d, M, D, device=dev)
    _lib.set_decode_shape(shape)
    try:
        for _ in range(warmup):
            dec.loss_and_grads(Q, K, V, T, K, 0.1)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            dec.loss_and_grads(Q, K, V, T, K, 0.1)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
    finally:
        _lib.set_decode_shape("px32")
    return float(np.median(ts))


def best_decode_shape(precision: str, n: int, d: int, M: int, D: int, use_cache: bool = True,
                      reps: int = 5) -> Tuple[str, dict]:
    """Fastest decode block shape for these sizes (it is not set; call
    ``_lib.set_decode_shape`` with the result)."""
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    key = f"{arch}|decode|{precision}|n={n}|d={d}|M={M}|D={D}"
    db = _load() if use_cache else {}
    if use_cache and key in db:
        return db[key]["shape"], db[key]["ms"]
    times = {s: time_decode_shape(precision, n, d, M, D, s, reps=reps) for s in _lib.DECODE_SHAPES}
    best = min(times, key=times.get)
    if use_cache:
        db[key] = {"shape": best, "ms": times}
        _store(db)
    return best, times
