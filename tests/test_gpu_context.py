"""The library context (lam_create / lam_destroy / lam_ctx_configure), the
autograd wrappers under HIP-graph capture, and the autotuner.

- options round-trip, bad options raise, a context is released once;
- two contexts with different launch options in one process each give
  exactly what they give alone (interleaved calls do not leak options);
- RenderQueries + DecodeLoss + backward captured in a HIP graph: every replay
  (with eager work and synchronisations between replays) reproduces the eager
  outputs; a second forward on the same renderer before backward raises;
- the autotuner picks among its candidates, its JSON cache round-trips, and
  tuned launches give the untuned results (bitwise for the render, to
  rounding for the decode).
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_12314_amd import scenes  # noqa: E402
from tests.gpu_helpers import rel_err, say, to_np  # noqa: E402

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2602_12314_amd import _lib, ops
    return _lib, ops


def _decode_inputs(seed, n, d, M, D):
    rng = np.random.default_rng(seed)
    f = lambda *s: torch.as_tensor(rng.standard_normal(s).astype(np.float32), device="cuda")
    Q, K, V = f(n, d), f(M, d), f(M, D)
    T = torch.nn.functional.normalize(f(n, D), dim=1)
    K0 = K + 0.01 * f(M, d)
    return Q, K, V, T, K0


def test_context_options_round_trip():
    _lib, _ = _mods()
    say("[ctx] options round trip")
    c = _lib.Context(options={"decode_shape": "px64", "decode_splits": 32, "raster_schedule": "per_tile"})
    assert c.options() == {"decode_shape": 1, "decode_splits": 32, "raster_schedule": 0}
    assert c.get("device") == torch.cuda.current_device()
    c.configure(raster_schedule="persistent")
    assert c.options() == {"decode_shape": 1, "decode_splits": 32, "raster_schedule": 1}
    with pytest.raises(_lib.LamError):
        c.configure(decode_splits=12)  # not a multiple of 8
    with pytest.raises(_lib.LamError):
        c.configure(bogus=1)
    assert c.options()["decode_splits"] == 32  # a rejected change leaves the options alone
    with pytest.raises(_lib.LamError):
        _lib.Context(options={"decode_shape": 5})
    c.close()
    c.close()  # released once


def test_two_contexts_match_single_context_runs():
    _lib, ops = _mods()
    n, d, M, D = 5000, 16, 256, 512
    say(f"[ctx] two contexts interleaved, bf16 n={n} d={d} M={M} D={D}")
    Q, K, V, T, K0 = _decode_inputs(1, n, d, M, D)
    opts = {"a": {"decode_shape": "px32", "decode_splits": 0}, "b": {"decode_shape": "px64", "decode_splits": 64}}

    def run(ctx):
        dec = ops.Decoder("bf16", n, d, M, D, ctx=ctx)
        loss, dQ, dK, dV = dec.loss_and_grads(Q, K, V, T, K0, 0.1)
        F = dec.forward(Q, K, V)
        torch.cuda.synchronize()
        return [to_np(x) for x in (loss, dQ, dK, dV, F)]

    alone = {}
    for k, o in opts.items():
        c = _lib.Context(options=o)
        alone[k] = run(c)
        c.close()
    ca, cb = _lib.Context(options=opts["a"]), _lib.Context(options=opts["b"])
    for ctx, k in ((ca, "a"), (cb, "b"), (ca, "a"), (cb, "b")):
        got = run(ctx)
        for x, y in zip(got, alone[k]):
            assert np.array_equal(x, y), k
    # the two option sets agree to rounding (a different split of a pixel's
    # sums can move a BF16 rounding of its softmax weights)
    for x, y in zip(alone["a"][1:], alone["b"][1:]):
        assert rel_err(x, y) < 1e-3
    # render: per-tile and persistent schedules in two live contexts, bitwise
    s = scenes.make_scene(scenes.spec(0), seed=0)
    g = ops.Gaussians.from_numpy(s)
    ra = ops.Renderer(s.cams, s.n, 16, ctx=_lib.Context(options={"raster_schedule": "per_tile"}))
    rb = ops.Renderer(s.cams, s.n, 16, ctx=_lib.Context(options={"raster_schedule": "persistent"}))
    Qa, Ta = ra.forward(g)
    Qb, Tb = rb.forward(g)
    assert np.array_equal(to_np(Qa), to_np(Qb)) and np.array_equal(to_np(Ta), to_np(Tb))


def _leaf_params(s):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").requires_grad_(True)
    return [f(s.means), f(s.log_scales), f(s.quats), f(s.opacity_logits), f(s.queries)]


def test_autograd_step_under_graph_capture():
    _lib, ops = _mods()
    sp = scenes.spec(0)
    s = scenes.make_scene(sp, seed=0)
    say(f"[ctx] autograd render + decode captured in a HIP graph ({sp.name})")
    params = _leaf_params(s)
    K = torch.as_tensor(s.K, device="cuda").requires_grad_(True)
    V = torch.as_tensor(s.V, device="cuda").requires_grad_(True)
    K0 = torch.as_tensor(s.K0, device="cuda")
    tgt = torch.as_tensor(s.target, device="cuda")
    r = ops.Renderer(s.cams, s.n, sp.d)
    dec = ops.Decoder("bf16", sp.n_pixels, sp.d, sp.M, sp.D)
    leaves = params + [K, V]

    def step():
        Q, _ = ops.RenderQueries.apply(r, *params)
        loss = ops.DecodeLoss.apply(Q, K, V, K0, tgt, sp.lambda_tr, dec)
        loss.backward()
        return loss

    def grads():
        return [to_np(t.grad) for t in leaves]

    for t in leaves:
        t.grad = None
    eager_loss = float(step())
    eager = grads()
    assert r._fitted
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            for t in leaves:
                t.grad = None
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for t in leaves:
        t.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        static_loss = step()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        r.verify()  # the replay stayed inside the pair capacity
        assert float(static_loss) == eager_loss, rep
        got = grads()
        # the decode gradients and queries' path are deterministic; the
        # per-Gaussian sums of the render backward use float atomics
        for k, (x, y) in enumerate(zip(got, eager)):
            assert rel_err(x, y) < (1e-5 if k < 5 else 1e-6), (rep, k)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk


def test_render_backward_after_another_forward_raises():
    _lib, ops = _mods()
    sp = scenes.spec(0)
    s = scenes.make_scene(sp, seed=0)
    params = _leaf_params(s)
    r = ops.Renderer(s.cams, s.n, sp.d)
    Q1, _ = ops.RenderQueries.apply(r, *params)
    Q2, _ = ops.RenderQueries.apply(r, *params)  # overwrites the workspace Q1's backward needs
    with pytest.raises(RuntimeError, match="another forward"):
        Q1.sum().backward()
    Q2.sum().backward()  # the latest forward is fine
    assert params[0].grad is not None


def test_autotuner_candidates_cache_and_results(tmp_path, monkeypatch):
    _lib, ops = _mods()
    from paper_2602_12314_amd import autotune as AT
    monkeypatch.setenv("LAM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sp = scenes.spec(0)
    s = scenes.make_scene(sp, seed=0)
    g = ops.Gaussians.from_numpy(s)
    cands = ((16, 16), (8, 8), (32, 4))
    say("[autotune] tile and decode options on the 80x60 scene")
    tile, times = AT.best_tile(g, s.cams, candidates=cands, reps=2)
    assert tile in cands and set(times) == {f"{a}x{b}" for a, b in cands}
    db = json.load(open(tmp_path / "tune.json"))
    assert any(v.get("tile") == list(tile) for v in db.values())
    assert AT.best_tile(g, s.cams, candidates=cands, reps=2) == (tile, times)  # from the cache
    n, d, M, D = sp.n_pixels, sp.d, sp.M, sp.D
    cand_opts = AT.decode_candidates(splits=(0, 16))
    opts, dtimes = AT.best_decode_options("bf16", n, d, M, D, reps=2, candidates=cand_opts)
    assert opts in cand_opts and len(dtimes) == len(cand_opts)
    assert AT.best_decode_options("bf16", n, d, M, D, reps=2, candidates=cand_opts) == (opts, dtimes)
    assert json.loads(AT.options_json(opts)) == _lib._encode_options(opts)
    # tuned launches give the untuned results
    r0 = ops.Renderer(s.cams, s.n, d)
    rt = ops.Renderer(s.cams, s.n, d, tile=tile, ctx=_lib.Context(options=opts))
    Q0, T0 = r0.forward(g)
    Qt, Tt = rt.forward(g)
    assert np.array_equal(to_np(Q0), to_np(Qt)) and np.array_equal(to_np(T0), to_np(Tt))
    Q, K, V, T, K0 = _decode_inputs(2, n, d, M, D)
    base = ops.Decoder("bf16", n, d, M, D).loss_and_grads(Q, K, V, T, K0, 0.1)
    tuned = ops.Decoder("bf16", n, d, M, D, ctx=rt.ctx).loss_and_grads(Q, K, V, T, K0, 0.1)
    for x, y in zip(base, tuned):
        assert rel_err(to_np(y), to_np(x)) < 1e-3
