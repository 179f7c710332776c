"""Autotuner for the render tile shape and the decode launch options.

The rendered query map does not depend on the tile shape (each Gaussian is
blended into exactly the pixels of its footprint), so the shape is a pure
performance choice: ``best_tile`` times render forward + backward for each
candidate on the caller's own scene and cameras and keeps the fastest.
``best_decode_options`` times the decode + loss + gradients call for each
combination of the context options ``decode_shape`` (32 pixels x 4 waves, 64
pixels x 8 waves) and ``decode_splits`` (the dV GEMM's pixel-range splits) on
inputs of the caller's sizes, each under a context of its own; the results
agree to rounding.  The chosen options are what ``lam_create`` takes as its
JSON argument (``Context(options=...)``).  Results are cached in JSON keyed by
GPU architecture and workload shape (``$LAM_AUTOTUNE_CACHE``, default
``~/.cache/latentam/autotune.json``).
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Iterable, Optional, Tuple

import numpy as np
import torch

from . import _lib, ops

CANDIDATES = ((16, 16), (8, 8), (16, 8), (8, 16), (32, 8), (8, 32), (16, 4), (32, 4))
DECODE_SHAPES = tuple(_lib.DECODE_SHAPES)  # px32, px64
DECODE_SPLITS = (0, 16, 32, 64, 128)       # 0: the library's device-filling rule


def cache_path() -> str:
    return os.environ.get("LAM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "latentam", "autotune.json"))


def _arch() -> str:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _key(cams: np.ndarray, n_gauss: int, d: int) -> str:
    views = ",".join(f"{int(c[0])}x{int(c[1])}" for c in cams)
    return f"{_arch()}|N={n_gauss}|d={d}|views={views}"


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_tile(g: ops.Gaussians, cams, tile, reps: int = 5, warmup: int = 2, ctx=None) -> float:
    """Median ms of render forward + backward with a random upstream gradient."""
    r = ops.Renderer(cams, g.n, g.d, tile=tile, ctx=ctx)
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
              use_cache: bool = True, reps: int = 5, ctx=None) -> Tuple[Tuple[int, int], dict]:
    cams = np.asarray(cams, np.float32).reshape(-1, 22)
    key = _key(cams, g.n, g.d)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        ent = db[key]
        return tuple(ent["tile"]), ent["ms"]
    times = {f"{tw}x{th}": time_tile(g, cams, (tw, th), reps=reps, ctx=ctx) for tw, th in candidates}
    best = min(times, key=times.get)
    tile = tuple(int(v) for v in best.split("x"))
    if use_cache:
        db[key] = {"tile": list(tile), "ms": times}
        _store(db)
    return tile, times


def _decode_inputs(n, d, M, D):
    dev = torch.device("cuda", torch.cuda.current_device())
    gen = torch.Generator(device=dev).manual_seed(0)
    Q = torch.randn((n, d), device=dev, generator=gen)
    K = torch.randn((M, d), device=dev, generator=gen)
    V = torch.randn((M, D), device=dev, generator=gen)
    T = torch.nn.functional.normalize(torch.randn((n, D), device=dev, generator=gen), dim=1)
    return Q, K, V, T


def time_decode_options(precision: str, n: int, d: int, M: int, D: int, options: dict, reps: int = 5,
                        warmup: int = 2, inputs=None) -> float:
    """Median ms of decode + loss + gradients under a context with ``options``."""
    Q, K, V, T = inputs if inputs is not None else _decode_inputs(n, d, M, D)
    ctx = _lib.Context(options=options)
    dec = ops.Decoder(precision, n, d, M, D, device=Q.device, ctx=ctx)
    for _ in range(warmup):
        dec.loss_and_grads(Q, K, V, T, K, 0.1)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        dec.loss_and_grads(Q, K, V, T, K, 0.1)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    del dec
    ctx.close()
    return float(np.median(ts))


def decode_candidates(shapes=DECODE_SHAPES, splits=DECODE_SPLITS):
    return [{"decode_shape": s, "decode_splits": k} for s, k in itertools.product(shapes, splits)]


def _name(opt: dict) -> str:
    return f"{opt['decode_shape']}/splits={opt['decode_splits']}"


# A split count other than the library's own rule (0) is taken only when it is
# clearly faster.  Timed alone, the split counts of the dV GEMM differ by about
# the run-to-run noise (1-2 %), while in the training step the dV grid also sets
# how the dictionary gradients share the GPU with the compositing backward on
# the second stream, which this timing does not see.
SPLIT_TOL = 0.02


def pick_decode_options(cands, times: dict, tol: float = SPLIT_TOL) -> dict:
    """The fastest candidate, except that the fastest one with the library's
    split rule (decode_splits 0) wins when it is within ``tol`` of it."""
    t = lambda o: times[_name(o)]
    best = min(cands, key=t)
    rule = [o for o in cands if o["decode_splits"] == 0 and t(o) <= t(best) * (1.0 + tol)]
    return dict(min(rule, key=t)) if rule else dict(best)


def best_decode_options(precision: str, n: int, d: int, M: int, D: int, use_cache: bool = True,
                        reps: int = 5, candidates=None) -> Tuple[dict, dict]:
    """Fastest decode options for these sizes (see pick_decode_options):
    ({"decode_shape", "decode_splits"}, {candidate name: ms}).  Pass the
    options to ``Context(options=...)``."""
    key = f"{_arch()}|decode|{precision}|n={n}|d={d}|M={M}|D={D}"
    db = _load() if use_cache else {}
    if use_cache and key in db and "options" in db[key]:
        return dict(db[key]["options"]), db[key]["ms"]
    cands = candidates if candidates is not None else decode_candidates()
    inputs = _decode_inputs(n, d, M, D)
    times = {}
    for opt in cands:
        times[_name(opt)] = time_decode_options(precision, n, d, M, D, opt, reps=reps, inputs=inputs)
    best = pick_decode_options(cands, times)
    if use_cache:
        db[key] = {"options": dict(best), "ms": times}
        _store(db)
    return dict(best), times


def options_json(options: dict) -> str:
    """The JSON text ``lam_create`` takes for these options."""
    return json.dumps(_lib._encode_options(options), sort_keys=True)
