"""torch.autograd wrappers around the C ABI (memory, streams, autograd only).

- ``Renderer`` owns the render workspace for one camera set and tile shape and
  sizes its (Gaussian, tile) pair capacity from the library's own counters.
- ``RenderQueries.apply(renderer, means, log_scales, quats, opacity_logits,
  queries) -> (Q, T_final)``: Eq. 4, differentiable in the five inputs.
- ``DecodeLoss.apply(Q, K, V, K0, target, lambda_tr, precision, decoder) -> loss``:
  Eq. 5-6; the library computes the loss and its gradients in one call.
- ``Decode.apply(Q, K, V, precision, decoder) -> F``: Eq. 5 alone.
- ``TiedDecoder``: the paper's tied decode and full feature loss (Eq. 5-6:
  cosine logits of Q W against the atoms D at temperature tau, V = D, and the
  cosine, L2 and hinge trust-region terms) with gradients to Q, W and D.
- ``Renderer.forward_rgbd`` / ``backward_rgbd``, ``rgbd_l1_loss`` and
  ``ssim_loss``: colour and depth blended in the same pass as the queries
  (Sec. III-A), the L1 colour and depth terms and the SSIM term of the mapping
  objective (Eq. 7-9).
- ``StreamKMeans``: the dictionary initialisation of Eq. 10 (weighted
  micro-centres of the keyframe's embeddings, merged with the weighted global
  centres and re-clustered to K), plus plain ``assign`` / ``lloyd`` calls.
- ``stage2(decoder, Q, K, V, target, K0, lambda_tr, iters, step)``: the
  decode-only iterations of Alg. 1 Stage II (Gaussians, hence Q, fixed): each
  iteration is one library call computing the loss, dK and dV without dQ.
Every step of the method runs in the HIP library; nothing here computes it.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib


@dataclass
class Gaussians:
    means: torch.Tensor           # [N,3]
    log_scales: torch.Tensor      # [N,3]
    quats: torch.Tensor           # [N,4] (w, x, y, z)
    opacity_logits: torch.Tensor  # [N]
    queries: torch.Tensor         # [N,d]

    @classmethod
    def from_numpy(cls, scene, device="cuda") -> "Gaussians":
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)
        return cls(f(scene.means), f(scene.log_scales), f(scene.quats), f(scene.opacity_logits),
                   f(scene.queries))

    def zeros_like(self) -> "Gaussians":
        return Gaussians(*[torch.zeros_like(t) for t in self.tensors()])

    def tensors(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.queries)

    @property
    def n(self) -> int:
        return self.means.shape[0]

    @property
    def d(self) -> int:
        return self.queries.shape[1]


def _contig(t):
    t = t.detach()
    assert t.dtype == torch.float32 and t.is_cuda, "expects float32 CUDA/HIP tensors"
    return t.contiguous()


class Renderer:
    """Render workspace for a fixed camera set, Gaussian count and tile shape.

    The (Gaussian, tile) pair capacity is sized from the library's own counter:
    a forward reads it back (a host synchronisation) until one forward has
    fitted (``check="first"``, the default), or on every forward
    (``check="always"``).  Later forwards only enqueue work, so a step can be
    captured in a HIP graph; ``verify()`` reads the overflow flag of the last
    forward outside the step.  Each forward bumps ``generation``: the state a
    backward reads is that of the latest forward."""

    def __init__(self, cams, n_gauss: int, d: int, tile=(16, 16), capacity: Optional[int] = None,
                 device="cuda", headroom: float = 1.15, check: str = "first", ctx=None):
        assert check in ("first", "always")
        self.cams = _lib._cams(cams)
        self.n_gauss, self.d = int(n_gauss), int(d)
        self.tile_w, self.tile_h = int(tile[0]), int(tile[1])
        self.device = torch.device(device)
        self.headroom = headroom
        self.check_mode = check
        self.ctx = ctx
        w = self.cams[:, 0].astype(np.int64)
        h = self.cams[:, 1].astype(np.int64)
        self.n_pixels = int((w * h).sum())
        self.capacity = 0
        self.ws = None
        self.generation = 0
        self._fitted = False
        self._alloc(capacity if capacity is not None else 0)

    def _alloc(self, capacity: int):
        nbytes = _lib.render_workspace_size(self.n_gauss, self.d, self.cams, self.tile_w, self.tile_h,
                                            capacity, ctx=self.ctx)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        self.capacity = int(capacity)
        self._fitted = False

    def counters(self):
        """BLOCKING: (pairs needed, overflowed) of the last forward."""
        return _lib.render_counters(self.ws, ctx=self.ctx)

    def verify(self):
        """BLOCKING: raises if the last forward ran out of pair capacity (its
        output is then incomplete; the next checked forward re-sizes)."""
        need, over = self.counters()
        if over:
            self._fitted = False
            raise RuntimeError(f"render pair capacity {self.capacity} exceeded ({need} needed): "
                               "call forward(check=True) to re-size")
        return need

    def _checked(self, check) -> bool:
        if check is None:
            return self.check_mode == "always" or not self._fitted
        return bool(check)

    def forward(self, g: Gaussians, Q=None, T_final=None, check: Optional[bool] = None):
        if Q is None:
            Q = torch.empty((self.n_pixels, self.d), dtype=torch.float32, device=self.device)
        if T_final is None:
            T_final = torch.empty((self.n_pixels,), dtype=torch.float32, device=self.device)
        gg = Gaussians(*[_contig(t) for t in g.tensors()])
        check = self._checked(check)
        for _ in range(3):
            self.generation += 1
            _lib.render_forward(gg, self.cams, self.tile_w, self.tile_h, Q, T_final, self.ws,
                                self.capacity, ctx=self.ctx)
            if not check:
                break
            need, over = self.counters()
            if not over:
                self._fitted = True
                break
            self._alloc(int(need * self.headroom) + 4096)
        return Q, T_final

    def backward(self, g: Gaussians, dQ: torch.Tensor, out: Optional[Gaussians] = None) -> Gaussians:
        """Gradients for the upstream dQ of the latest forward (every output is
        overwritten)."""
        gg = Gaussians(*[_contig(t) for t in g.tensors()])
        if out is None:
            out = Gaussians(*[torch.empty_like(t) for t in gg.tensors()])
        _lib.render_backward(gg, self.cams, self.tile_w, self.tile_h, _contig(dQ), out, self.ws,
                             self.capacity, ctx=self.ctx)
        return out

    def forward_rgbd(self, g: Gaussians, colors, check: Optional[bool] = None):
        """Q, rgb [P, 3], depth [P], T_final: the query map with colour and depth
        blended in the same pass (Sec. III-A)."""
        P = self.n_pixels
        Q = torch.empty((P, self.d), dtype=torch.float32, device=self.device)
        rgb = torch.empty((P, 3), dtype=torch.float32, device=self.device)
        depth = torch.empty((P,), dtype=torch.float32, device=self.device)
        T_final = torch.empty((P,), dtype=torch.float32, device=self.device)
        gg = Gaussians(*[_contig(t) for t in g.tensors()])
        colors = _contig(colors)
        check = self._checked(check)
        for _ in range(3):
            self.generation += 1
            _lib.render_rgbd_forward(gg, colors, self.cams, self.tile_w, self.tile_h, Q, rgb, depth, T_final,
                                     self.ws, self.capacity, ctx=self.ctx)
            if not check:
                break
            need, over = self.counters()
            if not over:
                self._fitted = True
                break
            self._alloc(int(need * self.headroom) + 4096)
        return Q, rgb, depth, T_final

    def backward_rgbd(self, g: Gaussians, colors, dQ, d_rgb, d_depth):
        """Gradients (Gaussians, d_colors) for upstream dQ, d_rgb, d_depth."""
        gg = Gaussians(*[_contig(t) for t in g.tensors()])
        out = Gaussians(*[torch.empty_like(t) for t in gg.tensors()])
        d_colors = torch.empty((self.n_gauss, 3), dtype=torch.float32, device=self.device)
        _lib.render_rgbd_backward(gg, _contig(colors), self.cams, self.tile_w, self.tile_h, _contig(dQ),
                                  _contig(d_rgb), _contig(d_depth), out, d_colors, self.ws, self.capacity,
                                  ctx=self.ctx)
        return out, d_colors

    def debug_views(self):
        return _lib.render_debug_views(self.ws, self.n_gauss, self.d, self.cams, self.tile_w,
                                       self.tile_h, self.capacity, ctx=self.ctx)


class RenderQueries(torch.autograd.Function):
    """Eq. 4 as an autograd function.  The backward reads the tile lists and
    per-pixel state the forward left in the renderer's workspace, so another
    forward on the same renderer in between is an error (raised, not silently
    wrong).  After the renderer's capacity has fitted once, neither pass
    synchronises with the host."""

    @staticmethod
    def forward(ctx, renderer: Renderer, means, log_scales, quats, opacity_logits, queries):
        g = Gaussians(means, log_scales, quats, opacity_logits, queries)
        Q, T = renderer.forward(g)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, queries)
        ctx.mark_non_differentiable(T)
        return Q, T

    @staticmethod
    def backward(ctx, dQ, dT):
        if ctx.renderer.generation != ctx.generation:
            raise RuntimeError("RenderQueries.backward: the renderer ran another forward after this one, "
                               "so its workspace no longer holds this forward's state; use one Renderer per "
                               "differentiable render in flight")
        g = Gaussians(*ctx.saved_tensors)
        gr = ctx.renderer.backward(g, dQ)
        return (None,) + gr.tensors()


class Decoder:
    """Decode workspace for fixed (precision, n, d, M, D)."""

    def __init__(self, precision: str, n: int, d: int, M: int, D: int, device="cuda", ctx=None):
        self.precision = precision
        self.shape = (int(n), int(d), int(M), int(D))
        self.ctx = ctx
        nbytes = _lib.decode_workspace_size(precision, n, d, M, D, ctx=ctx)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.device = torch.device(device)

    def loss_and_grads(self, Q, K, V, target, K0, lambda_tr, want_dQ=True, row_cos=None, dict_stream=None):
        """Loss and gradients (Eq. 5-6).  With ``dict_stream`` (a torch stream)
        the dictionary gradients and the loss are computed there, beside what
        the caller queues next on the current stream; join the streams before
        reading loss, dK, dV or changing the inputs."""
        n, d, M, D = self.shape
        dev = self.device
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        dQ = torch.empty((n, d), dtype=torch.float32, device=dev) if want_dQ else None
        dK = torch.empty((M, d), dtype=torch.float32, device=dev)
        dV = torch.empty((M, D), dtype=torch.float32, device=dev)
        args = (_contig(Q), _contig(K), _contig(V), _contig(target), None if K0 is None else _contig(K0))
        if dict_stream is None:
            _lib.decode_loss(self.precision, *args, lambda_tr, loss, dQ, dK, dV, row_cos, self.ws, ctx=self.ctx)
        else:
            _lib.decode_loss_overlap(self.precision, *args, lambda_tr, loss, dQ, dK, dV, row_cos, self.ws,
                                     dict_stream.cuda_stream, ctx=self.ctx)
            for t in (loss, dK, dV, self.ws) + tuple(a for a in args if a is not None):
                t.record_stream(dict_stream)
        return loss, dQ, dK, dV

    def forward(self, Q, K, V, F=None):
        n, d, M, D = self.shape
        if F is None:
            F = torch.empty((n, D), dtype=torch.float32, device=self.device)
        _lib.decode_forward(self.precision, _contig(Q), _contig(K), _contig(V), F, self.ws, ctx=self.ctx)
        return F

    def backward(self, Q, K, V, dF, want_dQ=True):
        n, d, M, D = self.shape
        dQ = torch.empty((n, d), dtype=torch.float32, device=self.device) if want_dQ else None
        dK = torch.empty((M, d), dtype=torch.float32, device=self.device)
        dV = torch.empty((M, D), dtype=torch.float32, device=self.device)
        _lib.decode_backward(self.precision, _contig(Q), _contig(K), _contig(V), _contig(dF), dQ, dK,
                             dV, self.ws, ctx=self.ctx)
        return dQ, dK, dV


class DecodeLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q, K, V, K0, target, lambda_tr: float, decoder: Decoder):
        loss, dQ, dK, dV = decoder.loss_and_grads(Q, K, V, target, K0, lambda_tr,
                                                  want_dQ=Q.requires_grad)
        ctx.save_for_backward(*(t for t in (dQ, dK, dV) if t is not None))
        ctx.has_dQ = dQ is not None
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        saved = list(ctx.saved_tensors)
        dQ = saved.pop(0) if ctx.has_dQ else None
        dK, dV = saved
        s = gl
        return (None if dQ is None else dQ * s, dK * s, dV * s, None, None, None, None)


class Decode(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q, K, V, decoder: Decoder):
        ctx.save_for_backward(Q, K, V)
        ctx.decoder = decoder
        return decoder.forward(Q, K, V)

    @staticmethod
    def backward(ctx, dF):
        Q, K, V = ctx.saved_tensors
        dQ, dK, dV = ctx.decoder.backward(Q, K, V, dF)
        return dQ, dK, dV, None


def stage2(decoder: Decoder, Q, K, V, target, K0, lambda_tr: float, iters: int = 5, step=None):
    """Alg. 1 Stage II: ``iters`` (R2 in the paper, 5) decode-only iterations on a
    fixed query map ``Q`` (the pixels of all 1 + B views of the step, stacked).
    Each iteration is one ``lam_decode_loss`` call without dQ, which returns
    the loss, dK and dV; ``step(dK, dV)`` then updates the dictionary in place
    (the caller's optimiser).  Returns the loss of every iteration (device)."""
    losses = []
    for _ in range(iters):
        loss, _, dK, dV = decoder.loss_and_grads(Q, K, V, target, K0, lambda_tr, want_dQ=False)
        losses.append(loss)
        if step is not None:
            step(dK, dV)
    return torch.cat(losses)


# the paper's weights (Sec. IV); it gives no temperature, 0.1 is this library's reading
PAPER_TIED_PARAMS = dict(tau=0.1, lambda_cos=0.5, lambda_2=0.5, lambda_D=0.2, delta=0.1)


class TiedDecoder:
    """Workspace for the tied decode of n pixel rows (query dimension ds, M atoms,
    feature dimension df)."""

    def __init__(self, precision: str, n: int, ds: int, M: int, df: int, device="cuda", ctx=None):
        self.precision = precision
        self.shape = (int(n), int(ds), int(M), int(df))
        self.ctx = ctx
        nbytes = _lib.decode_tied_workspace_size(precision, n, ds, M, df, ctx=ctx)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.device = torch.device(device)

    def loss_and_grads(self, Q, W, D, target, D0, params=None, want_dQ=True):
        n, ds, M, df = self.shape
        dev = self.device
        params = dict(PAPER_TIED_PARAMS, **(params or {}))
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        dQ = torch.empty((n, ds), dtype=torch.float32, device=dev) if want_dQ else None
        dW = torch.empty((ds, df), dtype=torch.float32, device=dev)
        dD = torch.empty((M, df), dtype=torch.float32, device=dev)
        _lib.decode_tied_loss(self.precision, _contig(Q), _contig(W), _contig(D), _contig(target), _contig(D0),
                              params, loss, dQ, dW, dD, self.ws, ctx=self.ctx)
        return loss, dQ, dW, dD


PAPER_RGBD_WEIGHTS = dict(lambda_rgb=0.2, lambda_depth=0.1, lambda_ssim=0.8)  # lambda_I1, lambda_d, lambda_I2


def rgbd_l1_loss(rgb, rgb_obs, depth, depth_obs, lambda_rgb=0.2, lambda_depth=0.1, ctx=None):
    """(loss, d_rgb, d_depth) of the L1 colour and depth terms (Eq. 7-9)."""
    rgb, rgb_obs, depth, depth_obs = (_contig(t) for t in (rgb, rgb_obs, depth, depth_obs))
    dev = rgb.device
    ws = torch.empty(_lib.rgbd_l1_workspace_size(depth.shape[0], ctx=ctx), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    d_rgb = torch.empty_like(rgb)
    d_depth = torch.empty_like(depth)
    _lib.rgbd_l1_loss(rgb, rgb_obs, depth, depth_obs, lambda_rgb, lambda_depth, loss, d_rgb, d_depth, ws, ctx=ctx)
    return loss, d_rgb, d_depth


def ssim_loss(rgb, rgb_obs, cams, lam=0.8, d_rgb=None, ctx=None):
    """(loss, d_rgb) of lam (1 - SSIM) (Eq. 7); with d_rgb given the gradient is
    added to it (e.g. after rgbd_l1_loss)."""
    rgb, rgb_obs = _contig(rgb), _contig(rgb_obs)
    ws = torch.empty(_lib.ssim_workspace_size(cams, ctx=ctx), dtype=torch.uint8, device=rgb.device)
    loss = torch.empty(1, dtype=torch.float32, device=rgb.device)
    acc = d_rgb is not None
    if d_rgb is None:
        d_rgb = torch.empty_like(rgb)
    _lib.ssim_loss(rgb, rgb_obs, cams, lam, loss, d_rgb, acc, ws, ctx=ctx)
    return loss, d_rgb


MICRO_FACTOR = 5  # micro-centres per global centre (the paper's "5 by default")


class StreamKMeans:
    """Streaming K-means state: global centres D [Kp, D] and weights W [Kp]
    (empty until the first keyframe), K the dictionary size.

    ``step(F, seeds=None, m=None)`` summarises the keyframe's embeddings F [n, D]
    into m micro-centres (default min(n, MICRO_FACTOR K)) started at F[seeds]
    (default: a seeded random draw of m distinct rows), merges them with the
    global centres and re-clusters to K; returns the new (D, W)."""

    def __init__(self, precision: str, K: int, dim: int, iters_local: int = 10, iters_global: int = 10,
                 seed: int = 0, device="cuda", ctx=None):
        self.precision = precision
        self.ctx = ctx
        self.K, self.dim = int(K), int(dim)
        self.iters_local, self.iters_global = int(iters_local), int(iters_global)
        self.device = torch.device(device)
        self.rng = np.random.default_rng(seed)
        self.D = torch.zeros((0, dim), dtype=torch.float32, device=self.device)
        self.W = torch.zeros(0, dtype=torch.float32, device=self.device)
        self._ws = None

    def _workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def step(self, F, seeds=None, m: Optional[int] = None):
        F = _contig(F)
        n = F.shape[0]
        Kp = self.D.shape[0]
        if m is None:
            m = min(n, MICRO_FACTOR * self.K)
        if seeds is None:
            seeds = self.rng.choice(n, size=m, replace=False) if m > 0 else np.zeros(0, np.int64)
        seeds = np.asarray(seeds, dtype=np.int32)
        ws = self._workspace(_lib.stream_kmeans_workspace_size(self.precision, n, self.dim, Kp, self.K, len(seeds),
                                                               ctx=self.ctx))
        D_out = torch.empty((self.K, self.dim), dtype=torch.float32, device=self.device)
        W_out = torch.empty(self.K, dtype=torch.float32, device=self.device)
        _lib.stream_kmeans(self.precision, F, self.D if Kp else None, self.W if Kp else None, self.K, seeds,
                           self.iters_local, self.iters_global, D_out, W_out, ws, ctx=self.ctx)
        self.D, self.W = D_out, W_out
        return D_out, W_out


def kmeans_assign(precision: str, X, C, ctx=None):
    """Nearest centre (int32) and squared distance of every row of X."""
    X, C = _contig(X), _contig(C)
    ws = torch.empty(max(_lib.kmeans_workspace_size(precision, X.shape[0], X.shape[1], C.shape[0], ctx=ctx), 256),
                     dtype=torch.uint8, device=X.device)
    a = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    d2 = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _lib.kmeans_assign(precision, X, C, a, d2, ws, ctx=ctx)
    return a, d2


def kmeans_lloyd(precision: str, X, C0, iters: int, weights=None, ctx=None):
    """``iters`` Lloyd iterations from C0: (C, W, last assignment)."""
    X, C0 = _contig(X), _contig(C0)
    ws = torch.empty(max(_lib.kmeans_workspace_size(precision, X.shape[0], X.shape[1], C0.shape[0], ctx=ctx), 256),
                     dtype=torch.uint8, device=X.device)
    C = torch.empty_like(C0)
    W = torch.empty(C0.shape[0], dtype=torch.float32, device=X.device)
    a = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    _lib.kmeans_lloyd(precision, X, None if weights is None else _contig(weights), C0, iters, C, W, a, ws, ctx=ctx)
    return C, W, a
