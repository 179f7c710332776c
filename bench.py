#!/usr/bin/env python3
"""Throughput of the render + decode hot path (forward and backward).

One step = render_forward (projection, binning, sort, compositing) + the
decode/loss call (softmax(Q K^T / sqrt d) V, cosine loss with trust region,
and its gradients) + render_backward.  The headline workload is the largest
single-GPU one: one 1200x680 keyframe of a 2M-Gaussian multi-floor map,
d = 32, M = D = 1024, decoded with E4M3 weights and V (the precision that
workload prescribes, and the fastest path that meets the error bar on it:
the product F = P V in E4M3, the logits and every backward product in BF16,
FP32 accumulation and softmax); the BF16 and FP32 decode paths are timed
beside it, and the
640x480 keyframe (100k Gaussians, d = 16, M = 256, D = 512), the 1200x680
keyframe of a 300k-Gaussian hall (d = 32, M = 512, D = 768) and the eight
keyframes of uneven size over a 500k-Gaussian local map (one launch per stage)
are secondary workloads.  Inputs are seeded synthetic arrays resident in HBM before timing
starts; the render tile shape and the decode block shape are autotuned.

Prints one JSON line: feature-pixels/s, per-stage times, the roofline of the
dominant kernel (timed with HIP events on its launch stream) against the
algorithmic work of the method, the error of every output against the FP64
oracle on the workload's 128 x 128 crop, and the FP64 CPU oracle timed on
the host.
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
    # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz: the library is built with
    # packed FP32 disabled, so the packed rate (twice this) is out of reach
    "fp32_vector_tflops": 78.6,
}

# the benchmark spec bars for the reduced-precision decode forms
BAR_MIN_COS_F = 0.999
BAR_GRAD_REL = 1e-2


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def decode_work(n, d, M, D):
    """Algorithmic work of the decode per launch (the method's, not the design's):
    per pixel 6 M (d + D) flops for S, F, dP, dV, dQ, dK, and (2 d + D) 4 bytes
    (Q and the target read once, dQ written once).  The rows kernel does S, F,
    dP and dQ (4 M (d + D)) and moves all of the per-pixel bytes; the dV kernel
    does 2 M D; the dK kernel 2 M d."""
    # e4m3_flops: the share that the E4M3 decode runs on E4M3 operands (F = P V)
    return {
        "decode_rows": dict(flops=4.0 * n * M * (d + D), bytes=4.0 * n * (2 * d + D), mfma=True,
                            e4m3_flops=2.0 * n * M * D),
        "decode_tn": dict(flops=2.0 * n * M * D, bytes=4.0 * M * D, mfma=True, e4m3_flops=0.0),
        "decode_total": dict(flops=6.0 * n * M * (d + D), bytes=4.0 * n * (2 * d + D), mfma=True,
                             e4m3_flops=2.0 * n * M * D),
    }


def decode_issued(n, d, M, D, prec):
    """Bytes the design adds on top: the rows kernel writes G^T, dS^T, Q^T in the
    compute type and one row max per pixel, which the dV and dK GEMMs read back;
    the softmax logits are recomputed (2 M d flops per pixel in each of the
    three passes that need them)."""
    tb = 4 if prec == "fp32" else 2
    Mp = (M + 63) // 64 * 64
    inter = n * (tb * (D + Mp + 32) + 4.0)
    return {"intermediate_bytes_written": inter, "intermediate_bytes_read": inter,
            "issued_flops_rows": n * (4.0 * M * (d + D) + 4.0 * M * d),
            "issued_flops_dv": n * 2.0 * M * (D + d)}


def raster_work(spec, pairs_eval: int, pairs_blend: int, tile_pairs: int):
    """Algorithmic work of the compositing kernels: per evaluated pair 20 flops
    (offset, conic form, exp, opacity, clamp, transmittance), per blended pair
    2 d more forward and 45 + 9 d backward; bytes: the tile lists, the per-pixel
    outputs and the per-record gradients."""
    n, d = spec.n_pixels, spec.d
    N = spec.n_gauss * len(spec.cams)
    entry = 44 + 4 * d  # one tile-list entry: record id, rec0, rec1, footprint, query
    return {
        "raster_fwd": dict(flops=20.0 * pairs_eval + 2.0 * d * pairs_blend, mfma=False,
                           bytes=tile_pairs * entry + n * (4.0 * d + 12)),
        "raster_bwd": dict(flops=(45.0 + 9.0 * d) * pairs_blend, mfma=False,
                           bytes=tile_pairs * entry + n * (4.0 * d + 8) + N * (24.0 + 4 * d)),
    }


def roofline(work: dict, ms: float, prec: str) -> dict:
    """Which roof binds at the kernel's algorithmic intensity, and how close it is.
    The E4M3 decode runs only F = P V on E4M3 operands and its other products
    in BF16, so its roof is the blend of the two peaks that the same flops
    would take at full rate: flops / (e4m3 / 5.0 + rest / 2.5 PFLOP/s)."""
    if work["mfma"]:
        fpeak = {"bf16": PEAKS["bf16_tflops"], "fp8": PEAKS["bf16_tflops"]}.get(prec, PEAKS["fp32_mfma_tflops"])
        f8 = work.get("e4m3_flops", 0.0) if prec == "fp8" else 0.0
        if f8 > 0.0:
            t_peak = f8 / PEAKS["fp8_tflops"] + (work["flops"] - f8) / PEAKS["bf16_tflops"]
            fpeak = work["flops"] / t_peak
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


PROF_STAGES = ("raster_fwd", "raster_bwd", "decode_rows", "decode_tn", "render_sort", "preprocess",
               "preprocess_bwd")


class Workload:
    """One workload on the GPU: scene, dictionary, target, renderer, and the
    step (render forward, decode + loss + gradients, render backward)."""

    def __init__(self, idx, prec, dev, autotune=True, tile="16x16", options=None):
        import torch

        from paper_2602_12314_amd import _lib, ops, scenes
        self.torch, self.ops, self._lib = torch, ops, _lib
        self.spec = scenes.spec(idx)
        self.prec = prec
        self.dev = dev
        _log(f"[bench] generating workload {self.spec.name}")
        s = scenes.make_scene(self.spec, seed=0)
        self.s = s
        self.g = ops.Gaussians.from_numpy(s, device=dev)
        self.K = torch.as_tensor(s.K, device=dev)
        self.V = torch.as_tensor(s.V, device=dev)
        self.K0 = torch.as_tensor(s.K0, device=dev)
        self.tgt = torch.as_tensor(s.target, device=dev)
        sp = self.spec
        self.n = sp.n_pixels
        tw, th = (int(v) for v in tile.split("x"))
        self.tune = None
        self.options = dict(options) if options else {"decode_shape": "px32", "decode_splits": 0}
        if autotune:
            from paper_2602_12314_amd import autotune as AT
            t0 = time.perf_counter()
            (tw, th), tile_ms = AT.best_tile(self.g, s.cams)
            self.options, dec_ms = AT.best_decode_options(prec, self.n, sp.d, sp.M, sp.D)
            self.tune = {"tile_ms": tile_ms, "decode_options_ms": dec_ms, "seconds": time.perf_counter() - t0}
            _log(f"[bench] autotuned tile {tw}x{th}: {tile_ms}")
            _log(f"[bench] autotuned decode options {self.options}: {dec_ms}")
        # one library context carries the tuned launch options for every call
        self.ctx = _lib.Context(options=self.options)
        self.tile = f"{tw}x{th}"
        self.r = ops.Renderer(s.cams, sp.n_gauss, sp.d, tile=(tw, th), ctx=self.ctx)
        self.Q = torch.empty((self.n, sp.d), device=dev)
        self.T = torch.empty((self.n,), device=dev)
        self.grads = self.g.zeros_like()
        self.side = torch.cuda.Stream(device=dev)
        self.r.forward(self.g, self.Q, self.T, check=True)  # sizes the pair capacity
        torch.cuda.synchronize()

    def decoder(self, prec, n=None):
        sp = self.spec
        return self.ops.Decoder(prec, self.n if n is None else n, sp.d, sp.M, sp.D, device=self.dev, ctx=self.ctx)

    def make_step(self, dec, overlap):
        r, g, Q, T, K, V, tgt, K0, lam = (self.r, self.g, self.Q, self.T, self.K, self.V, self.tgt, self.K0,
                                          self.spec.lambda_tr)
        torch, side, grads = self.torch, self.side, self.grads

        def step():
            r.forward(g, Q, T, check=False)
            if overlap:
                loss, dQ, dK, dV = dec.loss_and_grads(Q, K, V, tgt, K0, lam, dict_stream=side)
                r.backward(g, dQ, out=grads)
                torch.cuda.current_stream().wait_stream(side)
            else:
                loss, dQ, dK, dV = dec.loss_and_grads(Q, K, V, tgt, K0, lam)
                r.backward(g, dQ, out=grads)
            return loss
        return step

    def timed(self, dec, steps, warmup, profile=True):
        """Eager launches on one stream (the per-kernel times are taken without a
        concurrent kernel): seconds per step, loss, per-stage ms."""
        torch = self.torch
        step = self.make_step(dec, overlap=False)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        need, over = self.r.counters()
        assert not over, "pair capacity overflow after warm-up"
        ctx = self.ctx
        if profile:
            ctx.profile_enable(True)
            for name in PROF_STAGES:
                ctx.profile_read(name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            loss = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = {}
        if profile:
            for name in PROF_STAGES:
                tot, cnt = ctx.profile_read(name)
                if cnt:
                    prof[name] = tot / cnt
            ctx.profile_enable(False)
        self.pairs = need
        return (t1 - t0) / steps, float(loss), prof

    def graph_timed(self, dec, steps, warmup, overlap):
        """Replays of the step captured in a HIP graph (dictionary gradients on a
        second stream inside the graph when ``overlap``)."""
        torch = self.torch
        holder = {}
        base = self.make_step(dec, overlap=overlap)

        def step():
            holder["loss"] = base()

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
        assert not self.r.counters()[1]
        return (t1 - t0) / steps, float(holder["loss"])


def crop_window(spec):
    """The error crop of camera 0: a 128 x 128 window at the image centre
    (x0, y0, w, h), clipped to smaller images."""
    cam = spec.cams[0]
    w, h = min(128, cam.width), min(128, cam.height)
    return (cam.width - w) // 2, (cam.height - h) // 2, w, h


def _crop_pixels(cams, crop):
    import numpy as np
    x0, y0, cw, ch = crop
    W = int(cams[0, 0])
    return ((np.arange(ch)[:, None] + y0) * W + (np.arange(cw)[None, :] + x0)).ravel()


def oracle_reference(wl, crop):
    """The FP64 oracle on the workload: the whole frame's render forward, the
    decode of the crop's rows, and the render adjoint of the whole frame for
    the oracle's dQ on the crop (zero elsewhere, and on pixels whose walk takes
    a threshold decision within FP32 reach of the threshold).  Returns the
    reference arrays and the oracle's own times (s)."""
    import numpy as np

    from oracle import decode_oracle as DO
    from oracle import raster as R
    s, sp = wl.s, wl.spec
    pix = _crop_pixels(s.cams, crop)
    g = R.Gaussians.of(s)
    t0 = time.perf_counter()
    f = R.render_forward(g, s.cams)
    t_fwd = time.perf_counter() - t0
    ok = f["margin"][pix] >= 1e-5
    tgt = s.target[pix].astype(np.float64)
    t0 = time.perf_counter()
    d_or = DO.loss_and_grads(f["Q"][pix], s.K, s.V, tgt, s.K0, sp.lambda_tr)
    t_dec = time.perf_counter() - t0
    up = np.zeros((wl.n, sp.d))
    up[pix[ok]] = d_or["dQ"][ok]
    t0 = time.perf_counter()
    b = R.render_backward(g, s.cams, up)
    t_bwd = time.perf_counter() - t0
    return dict(crop=crop, pix=pix, ok=ok, f=f, tgt=tgt, up=up, bwd=b, t_fwd=t_fwd, t_dec=t_dec, t_bwd=t_bwd,
                pairs_eval=int(f["n_pairs"].sum()), pairs_blend=int(f["n_blended"].sum()))


def decode_errors(F, row_cos, loss, dQ, dK, dV, ref):
    """Errors of a decode call on the crop rows against the oracle's: F as the
    per-row cosine with the FP64 F (minimum, 1st percentile, mean) and relative
    L2; loss; each gradient as relative L2 and the largest element error
    relative to the tensor's largest element."""
    import numpy as np

    def rel(a, b):
        a = a.detach().double().cpu().numpy() if hasattr(a, "detach") else np.asarray(a, np.float64)
        return {"rel_l2": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
                "max_elem": float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))}
    Fg = F.detach().double().cpu().numpy()
    Fr = ref["F"]
    cF = (Fg * Fr).sum(1) / np.maximum(np.linalg.norm(Fg, axis=1) * np.linalg.norm(Fr, axis=1), 1e-300)
    out = {"F_cos_min": float(cF.min()), "F_cos_p1": float(np.percentile(cF, 1)), "F_cos_mean": float(cF.mean()),
           "F": rel(Fg, Fr),
           "row_cos_max_abs_err": float(np.abs(row_cos.double().cpu().numpy() - ref["cos"]).max()),
           "loss_rel_err": abs(float(loss) - ref["loss"]) / abs(ref["loss"]),
           "dQ": rel(dQ, ref["dQ"]), "dK": rel(dK, ref["dK"]), "dV": rel(dV, ref["dV"])}
    grad_worst = max(out[k]["rel_l2"] for k in ("dQ", "dK", "dV"))
    out["meets_bar"] = bool(out["F_cos_min"] >= BAR_MIN_COS_F and grad_worst <= BAR_GRAD_REL)
    return out


def oracle_check(wl, ref, precs):
    """One more step outside every timed region: the GPU's render (the crop,
    and over the whole frame the contributor counts), its decode of the crop
    rows in each precision, and its render backward for the oracle's upstream
    gradient on the crop, against the FP64 oracle."""
    import numpy as np
    torch = wl.torch

    from oracle import decode_oracle as DO
    sp, pix, ok, f = wl.spec, ref["pix"], ref["ok"], ref["f"]
    wl.r.forward(wl.g, wl.Q, wl.T, check=False)
    torch.cuda.synchronize()
    sel = torch.as_tensor(pix, device=wl.dev)
    Qg = wl.Q[sel].double().cpu().numpy()
    Qo = f["Q"][pix]
    Tg = wl.T[sel].double().cpu().numpy()
    To = f["T_final"][pix]
    amb_all = f["margin"] < 1e-5
    out = {"crop": list(ref["crop"]), "pixels": int(len(pix)), "ambiguous_pixels": int((~ok).sum()),
           "render": {"Q_rel_l2": float(np.linalg.norm(Qg[ok] - Qo[ok]) / np.linalg.norm(Qo[ok])),
                      "Q_max_elem": float(np.abs(Qg[ok] - Qo[ok]).max() / np.abs(Qo[ok]).max()),
                      "T_final_rel_l2": float(np.linalg.norm(Tg[ok] - To[ok]) / np.linalg.norm(To[ok])),
                      "T_final_max_abs": float(np.abs(Tg[ok] - To[ok]).max()),
                      "frame_ambiguous_fraction": float(amb_all.mean())}}
    # decode on the crop rows; the oracle takes the GPU's Q promoted to FP64
    Qc = wl.Q[sel].contiguous()
    Tc = wl.tgt[sel].contiguous()
    dref = DO.loss_and_grads(Qg, wl.s.K, wl.s.V, ref["tgt"], wl.s.K0, sp.lambda_tr)
    out["decode"] = {}
    for prec in precs:
        dec = wl.decoder(prec, n=len(pix))
        rc = torch.empty(len(pix), device=wl.dev)
        loss, dQ, dK, dV = dec.loss_and_grads(Qc, wl.K, wl.V, Tc, wl.K0, sp.lambda_tr, row_cos=rc)
        F = dec.forward(Qc, wl.K, wl.V)
        torch.cuda.synchronize()
        out["decode"][prec] = decode_errors(F, rc, loss, dQ, dK, dV, dref)
        del dec
    # render backward for the oracle's upstream gradient on the crop
    up32 = torch.as_tensor(ref["up"].astype(np.float32), device=wl.dev)
    gr = wl.r.backward(wl.g, up32)
    torch.cuda.synchronize()
    rb = {}
    for name in ("means", "log_scales", "quats", "opacity_logits", "queries"):
        a = getattr(gr, name).double().cpu().numpy()
        b = ref["bwd"][name]
        rb["d_" + name] = {"rel_l2": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
                           "max_elem": float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))}
    out["render_backward"] = rb
    return out


def cpu_baseline(wl, ref):
    """The FP64 oracle step (render forward, decode + loss + gradients, render
    backward) timed on the host: the whole frame's render and render adjoint,
    and the decode of the crop's rows extrapolated per pixel to the frame; on
    all host threads, and on one thread over the Gaussians and pixels of a
    32 x 32 part of the crop, extrapolated per pixel."""
    from oracle import raster as R
    sp = wl.spec
    x0, y0, cw, ch = ref["crop"]
    npx = len(ref["pix"])
    full_s = ref["t_fwd"] + ref["t_bwd"] + ref["t_dec"] * wl.n / npx
    threads = R.num_threads()
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        blas = 1
    one = _one_thread_sample(wl, (x0 + cw // 2 - 16, y0 + ch // 2 - 16, 32, 32))
    return {"value": wl.n / full_s, "unit": "feature-pixels/s", "cores": max(threads, blas), "kind": "oracle",
            "sample": (f"{sp.name}, whole frame ({wl.n} px, {sp.n_gauss} Gaussians): render fwd "
                       f"{ref['t_fwd']:.2f}s + render bwd {ref['t_bwd']:.2f}s; decode/loss/grads of the "
                       f"{cw}x{ch} crop's {npx} rows {ref['t_dec']:.2f}s, extrapolated per pixel: "
                       f"{full_s:.1f}s per step (C/OpenMP {threads} threads, numpy BLAS {blas} threads, FP64)"),
            "extrapolated": "decode part, per pixel", "one_thread": one, "host_cpu": _cpu_model(),
            "host_threads_visible": len(os.sched_getaffinity(0))}


def _one_thread_sample(wl, crop):
    """The oracle step on one thread for the pixels of a small crop: the
    projection of every Gaussian, then the Gaussians whose footprint overlaps
    the crop rendered, decoded and differentiated; extrapolated per pixel."""
    import numpy as np

    from oracle import decode_oracle as DO
    from oracle import raster as R
    s, sp = wl.s, wl.spec
    x0, y0, cw, ch = crop
    pix = _crop_pixels(s.cams, crop)
    prev = R.num_threads()
    lim = None
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=1)
    except Exception:
        pass
    R.set_num_threads(1)
    try:
        g = R.Gaussians.of(s)
        t0 = time.perf_counter()
        p = R.project(g, s.cams[:1])
        t_proj = time.perf_counter() - t0
        rect = p["rect"]
        ov = (p["vis"] == 1) & (rect[:, 0] <= x0 + cw - 1) & (rect[:, 1] >= x0) & \
             (rect[:, 2] <= y0 + ch - 1) & (rect[:, 3] >= y0)
        idx = np.nonzero(ov)[0]
        sub = R.Gaussians(*[np.ascontiguousarray(getattr(g, k)[idx]) for k in
                            ("means", "log_scales", "quats", "opacity_logits", "queries")])
        t0 = time.perf_counter()
        f = R.render_forward(sub, s.cams[:1])
        d = DO.loss_and_grads(f["Q"][pix], s.K, s.V, s.target[pix].astype(np.float64), s.K0, sp.lambda_tr)
        up = np.zeros((R.n_pixels(s.cams[:1]), sp.d))
        up[pix] = d["dQ"]
        R.render_backward(sub, s.cams[:1], up)
        t_crop = time.perf_counter() - t0
    finally:
        R.set_num_threads(prev)
        if lim is not None:
            lim.unregister()
    full_s = t_proj + t_crop * wl.n / len(pix)
    return {"value": wl.n / full_s, "unit": "feature-pixels/s", "cores": 1,
            "sample": f"projection of all Gaussians {t_proj:.2f}s, then the {cw}x{ch} crop at ({x0}, {y0}) "
                      f"with its {len(idx)} overlapping Gaussians {t_crop:.2f}s, extrapolated per pixel: "
                      f"{full_s:.1f}s per step"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run(args):
    import numpy as np
    import torch

    from paper_2602_12314_amd import _lib, ops

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    from paper_2602_12314_amd import scenes
    prec = args.precision or scenes.spec(args.workload).precision
    fixed = json.loads(args.decode_options) if args.decode_options else None
    wl = Workload(args.workload, prec, dev, autotune=not args.no_autotune, tile=args.tile, options=fixed)
    sp, n = wl.spec, wl.n

    dec = wl.decoder(prec)
    _log(f"[bench] timing {args.steps} steps ({prec} decode)")
    eager_sec, loss, prof = wl.timed(dec, args.steps, args.warmup, profile=True)
    sec = eager_sec
    if not args.eager:
        _log(f"[bench] timing {args.steps} HIP-graph replays ({prec} decode)")
        sec, loss = wl.graph_timed(dec, args.steps, args.warmup, overlap=not args.no_overlap)

    legs = {}
    for lp in ("bf16", "fp8", "fp32"):
        if lp == prec or lp in args.skip_precisions:
            continue
        d2 = wl.decoder(lp)
        st = max(3, args.steps // 4) if lp == "fp32" else args.steps
        _log(f"[bench] timing {st} steps ({lp} decode)")
        s2, l2, p2 = wl.timed(d2, st, 2, profile=True)
        legs[lp] = {"value": n / s2, "ms_per_step": s2 * 1e3, "launch": "eager",
                    "stage_ms": {k: round(v, 4) for k, v in p2.items()},
                    "speedup_of_headline_eager": s2 / eager_sec}
        del d2

    # roofline of the dominant kernel, from the method's algorithmic work
    check = cpu = None
    work = decode_work(n, sp.d, sp.M, sp.D)
    if not args.no_oracle:
        crop = crop_window(sp)
        _log(f"[bench] FP64 oracle: whole frame render, crop {crop} decode")
        ref = oracle_reference(wl, crop)
        work.update(raster_work(sp, ref["pairs_eval"], ref["pairs_blend"], wl.pairs))
        check = oracle_check(wl, ref, [prec] + [p for p in legs])
        for lp in legs:
            legs[lp]["oracle_crop"] = check["decode"][lp]
        for lp in ("bf16", "fp8"):
            if lp in legs:
                legs[lp]["bar"] = {"F_cos_min": BAR_MIN_COS_F, "grad_rel_l2": BAR_GRAD_REL}
                legs[lp]["bar_met"] = check["decode"][lp]["meets_bar"]
        if not args.no_cpu_baseline:
            _log("[bench] timing the FP64 CPU oracle (one thread)")
            cpu = cpu_baseline(wl, ref)
        del ref
    dom = max((k for k in prof if k in work), key=lambda k: prof[k])
    ms = prof[dom]
    rl = roofline(work[dom], ms, prec)
    dec_ms = sum(prof.get(k, 0.0) for k in ("decode_rows", "decode_tn"))
    out = {
        "metric": "feature-pixels/s fwd+bwd",
        "value": n / sec,
        "unit": "feature-pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "ms_per_keyframe": sec * 1e3 / len(sp.cams),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": sp.name, "n_gaussians": sp.n_gauss,
                   "image": f"{wl.s.cams[0, 0]:.0f}x{wl.s.cams[0, 1]:.0f}", "views": len(sp.cams),
                   "pixels": n, "d": sp.d, "M": sp.M, "D": sp.D, "decode_precision": prec,
                   "decode_arithmetic": {"fp8": "F = P V on E4M3 operands (V per-atom scaled, the weights as "
                                                "two E4M3 terms); logits and backward products in BF16; FP32 "
                                                "accumulation and softmax",
                                         "bf16": "all products on BF16 operands; FP32 accumulation and softmax",
                                         "fp32": "all products in FP32"}[prec],
                   "tile": wl.tile, "decode_options": wl.options, "tile_pairs": wl.pairs},
        "stage_ms": {k: round(v, 4) for k, v in prof.items()},
        "launch": "eager" if args.eager else "hip_graph_replay",
        "dict_gradients_on_second_stream": bool(not args.eager and not args.no_overlap),
        "eager_ms_per_step": eager_sec * 1e3,
        "autotune_ms": wl.tune,
        "loss": loss,
        "precision_legs": legs,
        "decode_error_bar": (None if check is None else
                             {"F_cos_min": BAR_MIN_COS_F, "grad_rel_l2": BAR_GRAD_REL,
                              "met": check["decode"][prec]["meets_bar"]}),
        "roofline": dict(kernel=dom, **rl, kernel_ms=ms, algorithmic_bytes=work[dom]["bytes"],
                         algorithmic_flops=work[dom]["flops"], traffic=traffic_for(dom, sp.name, {"tile": wl.tile, "precision": prec, **wl.options}),
                         issued=decode_issued(n, sp.d, sp.M, sp.D, prec) if dom.startswith("decode") else None),
        "decode_roofline": dict(**roofline(work["decode_total"], dec_ms, prec), ms=dec_ms,
                                kernels="decode_rows + decode_tn (+ dK GEMM and reductions not timed)"),
        "kernels": {k: dict(ms=round(prof[k], 4), **{kk: (round(vv, 4) if isinstance(vv, float) else vv)
                                                     for kk, vv in roofline(work[k], prof[k], prec).items()})
                    for k in work if k in prof},
        "oracle_check": check,
        "cpu_baseline": cpu,
    }
    if not args.no_extra_legs:
        out["stage2"] = stage2_leg(ops, dec, prec, sp, wl.Q, wl.K, wl.V, wl.tgt, wl.K0, dev, wl.ctx)
        out["tied_decode"] = tied_leg(ops, prec, sp, wl.Q, wl.V, wl.tgt, dev, wl.ctx)
        out["stream_kmeans"] = kmeans_leg(ops, prec, sp, wl.tgt, dev, wl.ctx)
        out["rgbd_step"] = rgbd_leg(ops, wl.r, wl.g, dec, wl.K, wl.V, wl.tgt, wl.K0, sp, dev, args.steps,
                                    side=None if args.no_overlap else wl.side)
    del dec
    sec_wl = {}
    for w2 in args.secondary:
        if w2 == args.workload:
            continue
        del wl
        torch.cuda.empty_cache()
        wl = Workload(w2, "bf16", dev, autotune=not args.no_autotune, tile=args.tile)
        d2 = wl.decoder("bf16")
        e2, _, p2 = wl.timed(d2, args.steps, args.warmup, profile=True)
        g2, _ = wl.graph_timed(d2, args.steps, args.warmup, overlap=not args.no_overlap)
        w2k = decode_work(wl.n, wl.spec.d, wl.spec.M, wl.spec.D)
        dom2 = max((k for k in p2 if k in w2k), key=lambda k: p2[k])
        sec_wl[wl.spec.name] = {"value": wl.n / g2, "ms_per_step": g2 * 1e3, "eager_ms_per_step": e2 * 1e3,
                                "views": len(wl.spec.cams), "pixels": wl.n,
                                "ms_per_keyframe": g2 * 1e3 / len(wl.spec.cams),
                                "decode_precision": "bf16", "tile": wl.tile, "decode_options": wl.options,
                                "stage_ms": {k: round(v, 4) for k, v in p2.items()},
                                "roofline": dict(kernel=dom2, **roofline(w2k[dom2], p2[dom2], "bf16"),
                                                 kernel_ms=p2[dom2],
                                                 traffic=traffic_for(dom2, wl.spec.name,
                                                                     {"tile": wl.tile, "precision": "bf16",
                                                                      **wl.options}))}
        del d2
    out["secondary_workloads"] = sec_wl
    print(json.dumps(out), flush=True)


def stage2_leg(ops, dec1, prec, spec, Q, K, V, tgt, K0, dev, ctx, views=6, iters=5, reps=3):
    """Alg. 1 Stage II on this workload: the query maps of 1 + B = 6 views
    (here the keyframe's own map six times; the decode cost depends only on the
    shapes) stay fixed while R2 = 5 decode-only iterations (loss, dK, dV; no dQ)
    update the dictionary with Adam."""
    import torch
    n = Q.shape[0] * views
    Q6 = Q.repeat(views, 1).contiguous()
    T6 = tgt.repeat(views, 1).contiguous()
    dec = ops.Decoder(prec, n, spec.d, spec.M, spec.D, device=dev, ctx=ctx)
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
    del Q6, T6, dec
    return {"views": views, "iters": iters, "pixels_per_iter": n, "ms": sec * 1e3,
            "value": n * iters / sec, "unit": "feature-pixels/s (decode + loss + dK, dV; Adam on K, V)",
            "loss_first_last": [float(losses[0]), float(losses[-1])]}


def tied_leg(ops, prec, spec, Q, V, tgt, dev, ctx, reps=10):
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
    dec = ops.TiedDecoder(prec, n, d, M, Dd, device=dev, ctx=ctx)
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
                                              w["lambda_depth"], ctx=r.ctx)
        ls, _ = ops.ssim_loss(rgb, rgb_obs, r.cams, w["lambda_ssim"], d_rgb=d_rgb, ctx=r.ctx)
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


def kmeans_leg(ops, prec, spec, tgt, dev, ctx, reps=3, iters=10):
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
        sk = ops.StreamKMeans(kprec, K, Dd, iters_local=iters, iters_global=iters, seed=r, device=dev, ctx=ctx)
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
    ws = torch.empty(_lib.kmeans_workspace_size(kprec, n, Dd, m, ctx=ctx), dtype=torch.uint8, device=dev)
    a = torch.empty(n, dtype=torch.int32, device=dev)
    _lib.kmeans_assign(kprec, tgt, C, a, None, ws, ctx=ctx)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ctx.profile_read("kmeans_assign")
    for _ in range(10):
        _lib.kmeans_assign(kprec, tgt, C, a, None, ws, ctx=ctx)
    torch.cuda.synchronize()
    tot, cnt = ctx.profile_read("kmeans_assign")  # the distance kernel alone, HIP events on its stream
    ctx.profile_enable(False)
    amsec = tot / max(cnt, 1)
    flops = 2.0 * n * m * Dd
    peak = PEAKS["fp32_mfma_tflops" if kprec == "fp32" else "bf16_tflops"]
    ach = flops / (amsec * 1e-3) / 1e12
    return {"ms": step_ms, "value": n / (step_ms * 1e-3), "unit": "embeddings/s (Eq. 10 streaming step)",
            "precision": kprec, "n": n, "D": Dd, "K": K, "micro": m, "iters_local": iters, "iters_global": iters,
            "assign": {"ms": amsec, "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                       "frac": ach / peak, "flops": flops, "bytes": 4.0 * n * Dd + 4.0 * n,
                       "traffic": traffic_for("kmeans_assign", spec.name)}}


def traffic_for(kernel, workload, options=None):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current sources of that kernel and, where the summary
    records them, with the same launch options; otherwise null."""
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
    # only the options that change the kernel's bytes must match: the decode
    # block shape for the rows kernel, also the split count for the dV partials,
    # the tile shape for the compositing kernels
    keys = {"decode_rows": ("precision", "decode_shape"),
            "decode_tn": ("precision", "decode_shape", "decode_splits"),
            "raster_fwd": ("tile",), "raster_bwd": ("tile",)}.get(kernel, ())
    rec_opts = ent.get("options") or {}
    if options is not None and any(k in rec_opts and rec_opts[k] != options.get(k) for k in keys):
        return None
    return ent.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=4,
                    help="0..4 (default 4: the 1200x680 keyframe of the 2M-Gaussian map)")
    ap.add_argument("--precision", default=None,
                    help="headline decode precision: bf16 | fp8 | fp32 (default: the workload's own, "
                         "fp8 for the 2M-Gaussian keyframe)")
    ap.add_argument("--skip-precisions", default="", help="comma list of precision legs to skip (bf16, fp8, fp32)")
    ap.add_argument("--secondary", default="1,2,3",
                    help="comma list of further workloads timed in BF16 (default: the 640x480 keyframe, the "
                         "1200x680 keyframe of the 300k-Gaussian hall, the eight keyframes of the local map)")
    ap.add_argument("--tile", default="16x16", help="render tile shape when not autotuned")
    ap.add_argument("--no-autotune", action="store_true", help="fixed tile and decode block shape")
    ap.add_argument("--decode-options", default=None, metavar="JSON",
                    help="decode launch options when not autotuned, e.g. "
                         "'{\"decode_shape\": \"px64\", \"decode_splits\": 0}' (default px32, no split)")
    ap.add_argument("--no-oracle", action="store_true", help="skip the FP64 oracle check and CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches instead of HIP-graph replays of the captured step")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the Stage-II, tied-decode, K-means and colour/depth legs")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the dictionary gradients on the step's own stream (no second stream)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (scales HBM byte counters)")
    args = ap.parse_args()
    args.skip_precisions = [p for p in args.skip_precisions.split(",") if p]
    args.secondary = [int(v) for v in args.secondary.split(",") if v != ""]
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
