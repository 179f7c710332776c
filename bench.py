#!/usr/bin/env python3
"""Throughput of the render + decode hot path (forward and backward).

One step = render_forward (projection, binning, sort, compositing) + the
decode/loss call (softmax(Q K^T / sqrt d) V, cosine loss with trust region,
and its gradients) + render_backward, for one keyframe of the 640x480
workload (100k Gaussians, d=16, M=256, D=512) with a BF16 decode.  Inputs
are seeded synthetic arrays resident in HBM before timing starts.

Prints one JSON line: feature-pixels/s, per-stage times, the roofline of the
dominant kernel (timed with HIP events on its launch stream), the FP32 decode
path for comparison, and the FP64 CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_gbs": 8000.0,
    "bf16_tflops": 2500.0,
    "fp8_tflops": 5000.0,
    "fp32_mfma_tflops": 157.3,
    "fp32_vector_tflops": 157.3,
}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_work(spec, prec: str, pairs_eval: int, pairs_blend: int, tile_pairs: int):
    """Algorithmic flops and HBM bytes per launch of each main kernel.

    Bytes count what the kernel must move to and from HBM once: its per-pixel
    inputs and outputs, the per-pair records of the tile lists, and the
    operands it hands to the next kernel.  The dictionary (K, V) is read from
    the L2 cache and counted once per launch.
    """
    n, d, M, D = spec.n_pixels, spec.d, spec.M, spec.D
    N = spec.n_gauss * len(spec.cams)
    Mp = (M + 63) // 64 * 64
    splits = dv_splits(n, Mp, D)
    tb = 4 if prec == "fp32" else 2  # bytes of the decode's compute type
    dict_bytes = tb * (2 * M * D + 2 * M * d)
    entry = 44 + 4 * d  # one tile-list entry: record id, rec0, rec1, footprint, query
    return {
        # MFMA: S = Q K^T (2Md), F = P V (2MD), dP = G V^T (2MD), dQ = dS K (2Md) per pixel.
        # Bytes: Q and the target in (FP32); G^T, dS^T, Q^T (compute type) and the
        # row max (FP32) out.
        "decode_rows": dict(flops=n * 4.0 * M * (d + D), mfma=True,
                            bytes=n * (4.0 * d + 4.0 * D + tb * (M + D + 32) + 4) + dict_bytes),
        # MFMA: dV = P~^T G with P~ rebuilt from S = Q K^T, 2M (D + d) per pixel;
        # bytes: G^T, Q and the row max in, the split partials out.
        "decode_tn": dict(flops=n * 2.0 * M * (D + d), mfma=True,
                          bytes=n * (tb * D + 4.0 * d + 4) + splits * Mp * D * 4.0),
        # VALU: per evaluated pair 20 flops (offset, conic form, exp, opacity, clamp,
        # transmittance); per blended pair 2d more for the query accumulation.
        # Bytes: the tile lists, and Q, T (twice) and the contributor count per pixel.
        "raster_fwd": dict(flops=20.0 * pairs_eval + 2.0 * d * pairs_blend, mfma=False,
                           bytes=tile_pairs * entry + n * (4.0 * d + 12)),
        # VALU: per blended pair 45 + 9d flops (alpha and transmittance rebuild,
        # dq, dalpha, behind-sum update, conic/mean/opacity terms).  Bytes: the tile
        # lists, dQ, T and the count per pixel, and the per-record gradients.
        "raster_bwd": dict(flops=(45.0 + 9.0 * d) * pairs_blend, mfma=False,
                           bytes=tile_pairs * entry + n * (4.0 * d + 8) + N * (24.0 + 4 * d)),
    }


def dv_splits(n: int, Mp: int, D: int) -> int:
    """Split-K count of the dV reduction (decode_layout's rule): enough
    workgroups to fill 256 CUs twice, a multiple of 8, at most the block count."""
    nb = max(((n + 63) // 64) * 2, 1)
    tiles = ((Mp + 127) // 128) * (D // (256 if D % 256 == 0 else 128))
    s = (512 + tiles - 1) // tiles
    s = (s + 7) // 8 * 8
    if s > nb:
        s = (nb + 7) // 8 * 8
    return max(s, 8)


def roofline(work: dict, ms: float, prec: str) -> dict:
    """Which roof binds at the kernel's algorithmic intensity, and how close it is."""
    if work["mfma"]:
        fpeak = {"bf16": PEAKS["bf16_tflops"], "fp8": PEAKS["fp8_tflops"]}.get(prec, PEAKS["fp32_mfma_tflops"])
    else:
        fpeak = PEAKS["fp32_vector_tflops"]
    t_flop = work["flops"] / (fpeak * 1e12)
    t_hbm = work["bytes"] / (PEAKS["hbm_gbs"] * 1e9)
    sec = ms * 1e-3
    if t_hbm >= t_flop:
        ach = work["bytes"] / sec / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
                "frac": ach / PEAKS["hbm_gbs"]}
    ach = work["flops"] / sec / 1e12
    return {"bound": "mfma" if work["mfma"] else "alu", "achieved": ach, "peak": fpeak,
            "unit": "TFLOP/s", "frac": ach / fpeak}


def run(args):
    import numpy as np
    import torch

    from paper_2602_12314_amd import _lib, ops, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    spec = scenes.spec(args.workload)
    prec = args.precision or spec.precision
    tw, th = (int(v) for v in args.tile.split("x"))
    _log(f"[bench] generating workload {spec.name}")
    s = scenes.make_scene(spec, seed=0)
    g = ops.Gaussians.from_numpy(s, device=dev)
    K = torch.as_tensor(s.K, device=dev)
    V = torch.as_tensor(s.V, device=dev)
    K0 = torch.as_tensor(s.K0, device=dev)
    tgt = torch.as_tensor(s.target, device=dev)
    n = spec.n_pixels
    tune = None
    if args.autotune:
        from paper_2602_12314_amd import autotune
        (tw, th), tune = autotune.best_tile(g, s.cams)
        args.tile = f"{tw}x{th}"
        _log(f"[bench] autotuned tile {args.tile}: {tune}")
    decode_shape = "px32"
    if args.autotune:
        from paper_2602_12314_amd import autotune
        decode_shape, dtimes = autotune.best_decode_shape(prec, n, spec.d, spec.M, spec.D)
        _lib.set_decode_shape(decode_shape)
        tune = {"tile_ms": tune, "decode_shape_ms": dtimes}
        _log(f"[bench] autotuned decode shape {decode_shape}: {dtimes}")
    r = ops.Renderer(s.cams, spec.n_gauss, spec.d, tile=(tw, th))
    Q = torch.empty((n, spec.d), device=dev)
    T = torch.empty((n,), device=dev)
    grads = g.zeros_like()

    # The dictionary gradients (dV, dK, their reductions, the loss) run on a
    # second stream beside the render backward, which needs only dQ.
    side = None if args.no_overlap else torch.cuda.Stream(device=dev)

    def make_step(dec, overlap=True):
        def step():
            r.forward(g, Q, T, check=False)
            if side is not None and overlap:
                loss, dQ, dK, dV = dec.loss_and_grads(Q, K, V, tgt, K0, spec.lambda_tr, dict_stream=side)
                r.backward(g, dQ, out=grads)
                torch.cuda.current_stream().wait_stream(side)
            else:
                loss, dQ, dK, dV = dec.loss_and_grads(Q, K, V, tgt, K0, spec.lambda_tr)
                r.backward(g, dQ, out=grads)
            return loss
        return step

    def timed(dec, steps, warmup, profile):
        # one stream: the per-kernel times are taken without a concurrent kernel
        step = make_step(dec, overlap=False)
        r.forward(g, Q, T, check=True)  # sizes the pair capacity
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        need, over = r.counters()
        assert not over, "pair capacity overflow after warm-up"
        L = _lib.lib()
        if profile:
            L.lam_profile_enable(1)
            for name in ("raster_fwd", "raster_bwd", "decode_rows", "decode_tn", "render_sort",
                         "preprocess", "preprocess_bwd"):
                _read_prof(L, name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            loss = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = {}
        if profile:
            for name in ("raster_fwd", "raster_bwd", "decode_rows", "decode_tn", "render_sort",
                         "preprocess", "preprocess_bwd"):
                tot, cnt = _read_prof(L, name)
                if cnt:
                    prof[name] = tot / cnt
            L.lam_profile_enable(0)
        return (t1 - t0) / steps, float(loss), prof, need

    def graph_timed(dec, steps, warmup):
        holder = {}
        base = make_step(dec, overlap=args.graph_overlap)

        def step():
            holder["loss"] = base()

        r.forward(g, Q, T, check=True)
        s_ = torch.cuda.Stream()
        s_.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_):
            for _ in range(max(1, warmup)):
                step()
        torch.cuda.current_stream().wait_stream(s_)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert not r.counters()[1]
        return (t1 - t0) / steps, float(holder["loss"])

    dec = ops.Decoder(prec, n, spec.d, spec.M, spec.D, device=dev)
    _log(f"[bench] timing {args.steps} steps ({prec} decode)")
    sec, loss, prof, pairs = timed(dec, args.steps, args.warmup, profile=True)
    eager_sec = sec
    if args.graph:
        _log(f"[bench] timing {args.steps} HIP-graph replays ({prec} decode)")
        sec, loss = graph_timed(dec, args.steps, args.warmup)
    if args.no_fp32 or prec == "fp32":
        sec32, prof32 = (sec, prof) if prec == "fp32" else (None, {})
    else:
        dec32 = ops.Decoder("fp32", n, spec.d, spec.M, spec.D, device=dev)
        fp32_steps = max(3, args.steps // 4)
        _log(f"[bench] timing {fp32_steps} steps (fp32 decode)")
        sec32, loss32, prof32, _ = timed(dec32, fp32_steps, 2, profile=True)
        del dec32

    stage2 = None
    if not args.no_stage2:
        stage2 = stage2_leg(ops, dec, prec, spec, Q, K, V, tgt, K0, dev)
    tied = None
    if not args.no_tied:
        tied = tied_leg(ops, prec, spec, Q, V, tgt, dev)
    kmeans = None
    if not args.no_kmeans:
        kmeans = kmeans_leg(ops, prec, spec, tgt, dev)
    rgbd = None
    if not args.no_rgbd:
        rgbd = rgbd_leg(ops, r, g, dec, K, V, tgt, K0, spec, dev, args.steps, side=side)

    out = {
        "metric": "feature-pixels/s fwd+bwd",
        "value": n / sec,
        "unit": "feature-pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "ms_per_keyframe": sec * 1e3 / len(spec.cams),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": spec.name, "n_gaussians": spec.n_gauss,
                   "image": f"{s.cams[0, 0]:.0f}x{s.cams[0, 1]:.0f}", "views": len(spec.cams),
                   "pixels": n, "d": spec.d, "M": spec.M, "D": spec.D, "decode_precision": prec,
                   "tile": args.tile, "decode_shape": decode_shape, "tile_pairs": pairs},
        "stage_ms": {k: round(v, 4) for k, v in prof.items()},
        "launch": "hip_graph_replay" if args.graph else "eager",
        "dict_gradients_on_second_stream": bool(args.graph and args.graph_overlap),
        "eager_ms_per_step": eager_sec * 1e3,
        "autotune_ms": tune,
        "loss": loss,
        "fp32_decode_path": None if sec32 is None else {
            "value": n / sec32, "ms_per_step": sec32 * 1e3,
            "stage_ms": {k: round(v, 4) for k, v in prof32.items()},
            "speedup_of_reduced_precision": sec32 / sec},
        "stage2": stage2,
        "tied_decode": tied,
        "stream_kmeans": kmeans,
        "rgbd_step": rgbd,
    }

    # roofline of the dominant kernel, with algorithmic work from the oracle's pair counts
    cpu = None
    pairs_eval = pairs_blend = None
    if not args.no_cpu_baseline:
        cpu, pairs_eval, pairs_blend, ref = cpu_baseline(s, spec)

        def check(prec_):
            # one more step, outside every timed region, against the oracle's FP64 step
            d_ = dec if prec_ == prec else ops.Decoder(prec_, n, spec.d, spec.M, spec.D, device=dev)
            r.forward(g, Q, T, check=False)
            l_, dQ_, dK_, dV_ = d_.loss_and_grads(Q, K, V, tgt, K0, spec.lambda_tr)
            gr_ = r.backward(g, dQ_)
            torch.cuda.synchronize()

            def rel(a, b):
                a = a.detach().double().cpu().numpy()
                return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
            return {"loss_rel_err": abs(float(l_) - ref["loss"]) / abs(ref["loss"]),
                    "dK_rel_err": rel(dK_, ref["dK"]), "dV_rel_err": rel(dV_, ref["dV"]),
                    "d_means_rel_err": rel(gr_.means, ref["means"]),
                    "d_queries_rel_err": rel(gr_.queries, ref["queries"])}
        out["oracle_check"] = {p_: check(p_) for p_ in dict.fromkeys([prec, "fp32"])}
    else:
        pairs_eval, pairs_blend = oracle_pairs(s)
    work = algorithmic_work(spec, prec, pairs_eval, pairs_blend, pairs)
    dom = max((k for k in prof if k in work), key=lambda k: prof[k])
    ms = prof[dom]
    rl = roofline(work[dom], ms, prec)
    out["roofline"] = dict(kernel=dom, **rl, kernel_ms=ms, algorithmic_bytes=work[dom]["bytes"],
                           algorithmic_flops=work[dom]["flops"], traffic=traffic_for(dom, spec.name))
    out["kernels"] = {k: dict(ms=round(prof[k], 4), **{kk: (round(vv, 4) if isinstance(vv, float) else vv)
                                                        for kk, vv in roofline(work[k], prof[k], prec).items()})
                      for k in work if k in prof}
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def stage2_leg(ops, dec1, prec, spec, Q, K, V, tgt, K0, dev, views=6, iters=5, reps=5):
    """Alg. 1 Stage II on this workload: the query maps of 1 + B = 6 views
    (here the keyframe's own map six times; the decode cost depends only on the
    shapes) stay fixed while R2 = 5 decode-only iterations (loss, dK, dV; no dQ)
    update the dictionary with Adam."""
    import torch
    n = Q.shape[0] * views
    Q6 = Q.repeat(views, 1).contiguous()
    T6 = tgt.repeat(views, 1).contiguous()
    dec = ops.Decoder(prec, n, spec.d, spec.M, spec.D, device=dev)
    Kp = torch.nn.Parameter(K.clone())
    Vp = torch.nn.Parameter(V.clone())
    opt = torch.optim.Adam([Kp, Vp], lr=1e-3)

    def step(dK, dV):
        Kp.grad, Vp.grad = dK, dV
        opt.step()

    def run():
        return ops.stage2(dec, Q6, Kp.data, Vp.data, T6, K0, spec.lambda_tr, iters=iters, step=step)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        losses = run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    return {"views": views, "iters": iters, "pixels_per_iter": n, "ms": sec * 1e3,
            "value": n * iters / sec, "unit": "feature-pixels/s (decode + loss + dK, dV; Adam on K, V)",
            "loss_first_last": [float(losses[0]), float(losses[-1])]}


def tied_leg(ops, prec, spec, Q, V, tgt, dev, reps=10):
    """The paper's tied decode (Eq. 5 with cosine logits at temperature 0.1,
    V = D) and full loss (cosine + L2 + hinge trust region, the paper's weights)
    with gradients to Q, W and D, on this workload's query map and shapes; W is
    a random d x D projection and D0 the dictionary before one perturbation.
    The library offers this form in FP32 and BF16 only, so an E4M3 workload
    runs it in BF16."""
    import torch
    n, d, M, Dd = spec.n_pixels, spec.d, spec.M, spec.D
    prec = "bf16" if prec == "fp8" else prec
    g = torch.Generator(device=dev).manual_seed(3)
    W = torch.randn((d, Dd), device=dev, generator=g) / d ** 0.5
    D0 = V.clone()
    Dm = D0 + 0.05 * torch.randn(D0.shape, device=dev, generator=g)
    dec = ops.TiedDecoder(prec, n, d, M, Dd, device=dev)
    dec.loss_and_grads(Q, W, Dm, tgt, D0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        loss, _, _, _ = dec.loss_and_grads(Q, W, Dm, tgt, D0)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    return {"ms": sec * 1e3, "value": n / sec, "unit": "feature-pixels/s (decode + loss + dQ, dW, dD)",
            "precision": prec, "params": dict(ops.PAPER_TIED_PARAMS), "loss": float(loss)}


def rgbd_leg(ops, r, g, dec, K, V, tgt, K0, spec, dev, steps, warmup=3, side=None):
    """The Stage-I step with colour and depth supervision (Eq. 7-9): query,
    colour and depth maps in one compositing pass, the decode with the feature
    loss, the L1 colour and depth terms and the SSIM term with the paper's
    weights, and one backward pass through queries, colour and depth.  Colours
    are seeded uniform; the observed image is uniform noise and the observed
    depth the rendered depth plus noise with 10 % holes."""
    import torch
    n = spec.n_pixels
    gen = torch.Generator(device=dev).manual_seed(11)
    colors = torch.rand((spec.n_gauss, 3), device=dev, generator=gen)
    _, rgb, depth, _ = r.forward_rgbd(g, colors)
    rgb_obs = torch.rand(rgb.shape, device=dev, generator=gen)
    depth_obs = depth + 0.05 * torch.randn(depth.shape, device=dev, generator=gen)
    depth_obs[torch.rand(depth.shape, device=dev, generator=gen) < 0.1] = 0.0
    w = ops.PAPER_RGBD_WEIGHTS

    def step():
        Q, rgb, depth, _ = r.forward_rgbd(g, colors, check=False)
        lf, dQ, _, _ = dec.loss_and_grads(Q, K, V, tgt, K0, spec.lambda_tr, dict_stream=side)
        lp, d_rgb, d_depth = ops.rgbd_l1_loss(rgb, rgb_obs, depth, depth_obs, w["lambda_rgb"],
                                              w["lambda_depth"])
        ls, _ = ops.ssim_loss(rgb, rgb_obs, r.cams, w["lambda_ssim"], d_rgb=d_rgb)
        r.backward_rgbd(g, colors, dQ, d_rgb, d_depth)
        if side is not None:
            torch.cuda.current_stream().wait_stream(side)
        return lf, lp + ls

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    assert not r.counters()[1]
    t0 = time.perf_counter()
    for _ in range(steps):
        lf, lp = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    return {"ms": sec * 1e3, "value": n / sec,
            "unit": "feature-pixels/s (queries, colour and depth rendered; feature, L1 colour/depth and SSIM losses)",
            "weights": dict(w), "loss_feature": float(lf), "loss_rgbd": float(lp)}


def kmeans_leg(ops, prec, spec, tgt, dev, reps=3, iters=10):
    """The streaming K-means dictionary initialisation (Eq. 10) on this
    workload's embedding map: m = 5 K micro-centres from seeded random rows,
    merged into K = M global centres (the previous dictionary: K rows of an
    earlier draw, weight 100 each), ``iters`` Lloyd iterations in each stage.
    Also the nearest-centre kernel alone (n x m x D distance GEMM) against the
    MFMA roof of its precision."""
    import numpy as np
    import torch
    from paper_2602_12314_amd import _lib
    kprec = "fp32" if prec == "fp32" else "bf16"
    n, Dd, K = tgt.shape[0], tgt.shape[1], spec.M
    m = min(n, ops.MICRO_FACTOR * K)
    rng = np.random.default_rng(5)
    prev = tgt[torch.as_tensor(rng.choice(n, K, replace=False), device=dev)].contiguous()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for r in range(reps + 1):
        sk = ops.StreamKMeans(kprec, K, Dd, iters_local=iters, iters_global=iters, seed=r, device=dev)
        sk.D, sk.W = prev, torch.full((K,), 100.0, device=dev)
        seeds = sk.rng.choice(n, size=m, replace=False)
        torch.cuda.synchronize()
        e0.record(st)
        sk.step(tgt, seeds=seeds)
        e1.record(st)
        torch.cuda.synchronize()
        if r > 0:
            ms.append(e0.elapsed_time(e1))
    step_ms = float(np.median(ms))
    C = tgt[torch.as_tensor(rng.choice(n, m, replace=False), device=dev)].contiguous()
    ws = torch.empty(_lib.kmeans_workspace_size(kprec, n, Dd, m), dtype=torch.uint8, device=dev)
    a = torch.empty(n, dtype=torch.int32, device=dev)
    _lib.kmeans_assign(kprec, tgt, C, a, None, ws)
    torch.cuda.synchronize()
    L = _lib.lib()
    L.lam_profile_enable(1)
    _read_prof(L, "kmeans_assign")
    for _ in range(10):
        _lib.kmeans_assign(kprec, tgt, C, a, None, ws)
    torch.cuda.synchronize()
    tot, cnt = _read_prof(L, "kmeans_assign")  # the distance kernel alone, HIP events on its stream
    L.lam_profile_enable(0)
    amsec = tot / max(cnt, 1)
    flops = 2.0 * n * m * Dd
    peak = PEAKS["fp32_mfma_tflops" if kprec == "fp32" else "bf16_tflops"]
    ach = flops / (amsec * 1e-3) / 1e12
    return {"ms": step_ms, "value": n / (step_ms * 1e-3), "unit": "embeddings/s (Eq. 10 streaming step)",
            "precision": kprec, "n": n, "D": Dd, "K": K, "micro": m, "iters_local": iters, "iters_global": iters,
            "assign": {"ms": amsec, "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                       "frac": ach / peak, "flops": flops, "bytes": 4.0 * n * Dd + 4.0 * n,
                       "traffic": traffic_for("kmeans_assign", spec.name)}}


def _read_prof(L, name):
    import ctypes as C
    tot, cnt = C.c_double(), C.c_int()
    L.lam_profile_read(name.encode(), C.byref(tot), C.byref(cnt))
    return tot.value, cnt.value


def traffic_for(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current sources of that kernel; otherwise null."""
    from paper_2602_12314_amd import profiling
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or kernel not in profiling.STAGES:
        return None
    if ent.get("source_hash") != profiling.source_hash(profiling.STAGES[kernel][1]):
        return None
    return ent.get("bytes_per_launch")


def oracle_pairs(s):
    from oracle import raster as R
    f = R.render_forward(R.Gaussians.of(s), s.cams)
    return int(f["n_pairs"].sum()), int(f["n_blended"].sum())


def cpu_baseline(s, spec):
    """The FP64 oracle (render forward, decode + loss + gradients, render
    backward) on the full frame, timed on the host cores."""
    import numpy as np

    from oracle import decode_oracle as DO
    from oracle import raster as R
    _log("[bench] timing the FP64 CPU oracle on the full frame")
    g = R.Gaussians.of(s)
    t0 = time.perf_counter()
    f = R.render_forward(g, s.cams)
    t1 = time.perf_counter()
    r = DO.loss_and_grads(f["Q"], s.K, s.V, s.target, s.K0, spec.lambda_tr)
    t2 = time.perf_counter()
    gb = R.render_backward(g, s.cams, r["dQ"])
    t3 = time.perf_counter()
    threads = R.num_threads()
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        blas = 1
    total = t3 - t0
    n = spec.n_pixels
    return ({"value": n / total, "unit": "feature-pixels/s", "cores": max(threads, blas),
             "kind": "oracle",
             "sample": f"one full {spec.name} step: render fwd {t1 - t0:.2f}s + decode/loss/grads "
                       f"{t2 - t1:.2f}s + render bwd {t3 - t2:.2f}s (C/OpenMP {threads} threads, "
                       f"numpy BLAS {blas} threads, FP64)"},
            int(f["n_pairs"].sum()), int(f["n_blended"].sum()),
            {"loss": float(r["loss"]), "dK": r["dK"], "dV": r["dV"], "means": gb["means"],
             "queries": gb["queries"]})


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=1, help="0..4 (default: the 640x480 keyframe)")
    ap.add_argument("--precision", default=None, help="decode precision: fp32 | bf16 (default: workload's)")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="pick the render tile shape by timing")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the HIP-graph-captured step (the default; see --eager)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches instead of HIP-graph replays of the captured step")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 decode comparison leg")
    ap.add_argument("--no-stage2", action="store_true", help="skip the Stage-II decode-only leg")
    ap.add_argument("--no-tied", action="store_true", help="skip the tied-decode leg")
    ap.add_argument("--no-kmeans", action="store_true", help="skip the streaming K-means leg")
    ap.add_argument("--no-rgbd", action="store_true", help="skip the colour + depth step leg")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the dictionary gradients on the step's own stream (no second stream)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (scales HBM byte counters)")
    args = ap.parse_args()
    args.graph = not args.eager
    args.graph_overlap = not args.no_overlap
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration // 4, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(every stage is per view and per pixel block, so views would be split across GPUs "
              "with one gradient all-reduce per step; that path is not built)", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
