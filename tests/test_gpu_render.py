"""GPU parity of the renderer (Eq. 2, Eq. 4 and their adjoint) against the FP64
oracle, through the C ABI.

- integer stage: per-record depth keys and footprints, the sorted (tile,
  record) list and the tile ranges must equal the oracle's bit for bit;
- Q and T_final within 1e-4 relative (FP32 kernel vs FP64 oracle) on every
  pixel whose oracle walk takes no threshold decision within 1e-5 of a
  threshold; contributor counts equal there; the ambiguous fraction is
  reported and bounded;
- gradients of <w, Q> for a seeded w (zeroed at ambiguous pixels) within
  1e-4 relative per tensor;
- Q is bitwise identical across tile shapes and across runs.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import raster as R  # noqa: E402
from paper_2602_12314_amd import scenes  # noqa: E402
from tests.gpu_helpers import AMBIGUOUS, rel_err, say, to_np, ws_u32  # noqa: E402
from tests.oracle_helpers import cams_of, gaussians, logit  # noqa: E402

pytestmark = pytest.mark.gpu


def _ops():
    from paper_2602_12314_amd import ops
    return ops


def _gpu_gauss(g):
    ops = _ops()
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    return ops.Gaussians(f(g.means), f(g.log_scales), f(g.quats), f(g.opacity_logits), f(g.queries))


def _scene(i, seed):
    s = scenes.make_scene(scenes.spec(i), seed=seed, with_target=False)
    return R.Gaussians.of(s), s.cams


def _small_multiview(seed=3):
    pose = scenes.look_at_origin((1.2, 0.0, -2.4))
    cams = cams_of(scenes.pinhole(70, 45, 50.0, pose), scenes.pinhole(37, 29, 30.0),
                   scenes.pinhole(64, 64, 60.0, scenes.look_at_origin((-2.0, 0.0, 1.0))))
    sp = scenes.custom_spec("mv", 3000, [scenes.pinhole(37, 29, 30.0)], d=16, box=((-1.5, 1.5), (-1, 1), (-1.5, 1.5)))
    s = scenes.make_scene(sp, seed=seed, with_target=False)
    g = R.Gaussians.of(s)
    g.means[:, 2] += 1.5  # keep some in front of the identity camera
    return g, cams


CASES = {
    "c0": lambda: _scene(0, 0),
    "c1": lambda: _scene(1, 1),
    "c2": lambda: _scene(2, 2),
    "multiview_ragged": _small_multiview,
}


def _render(g, cams, tile=(16, 16), d=None):
    ops = _ops()
    gg = _gpu_gauss(g)
    r = ops.Renderer(cams, g.n, g.d if d is None else d, tile=tile)
    Q, T = r.forward(gg)
    torch.cuda.synchronize()
    return r, gg, Q, T


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_binning_bit_exact(case, tile):
    if case == "c2" and tile != (16, 16):
        pytest.skip("full-size c2 checked at 16x16")
    g, cams = CASES[case]()
    say(f"[binning] case={case} tile={tile} N={g.n}")
    r, gg, Q, T = _render(g, cams, tile)
    need, over = r.counters()
    ob = R.bin_sort(g, cams, *tile)
    op = R.project(g, cams)
    assert not over and need == ob["count"]
    kp, rp, rgp, dkp, fpp, _ = r.debug_views()
    nrec = cams.shape[0] * g.n
    dk = ws_u32(r.ws, dkp, nrec)
    assert np.array_equal(dk, op["depth_key"]), "depth keys"
    fp = ws_u32(r.ws, fpp, 2 * nrec).reshape(-1, 2)
    vis = op["vis"] == 1
    rect = np.stack([fp[:, 0] & 0xFFFF, fp[:, 0] >> 16, fp[:, 1] & 0xFFFF, fp[:, 1] >> 16], 1)
    assert np.array_equal(rect[vis], op["rect"][vis].astype(np.uint32)), "footprints"
    keys = ws_u32(r.ws, kp, need)
    recs = ws_u32(r.ws, rp, need)
    assert np.array_equal(keys, ob["tiles"]), "tile keys"
    assert np.array_equal(recs, ob["recs"]), "record order"
    rg = ws_u32(r.ws, rgp, 2 * R.num_tiles(cams, *tile)).reshape(-1, 2)
    assert np.array_equal(rg, ob["ranges"]), "tile ranges"


@pytest.mark.parametrize("case", list(CASES))
def test_forward_parity(case):
    g, cams = CASES[case]()
    say(f"[forward] case={case} N={g.n}")
    r, gg, Q, T = _render(g, cams)
    ref = R.render_forward(g, cams)
    amb = ref["margin"] < AMBIGUOUS
    ok = ~amb
    frac = amb.mean()
    say(f"  ambiguous pixels {amb.sum()} ({frac:.2e})")
    assert frac < 0.01
    Qg, Tg = to_np(Q), to_np(T)
    eq = rel_err(Qg[ok], ref["Q"][ok])
    et = rel_err(Tg[ok], ref["T_final"][ok])
    say(f"  rel err Q {eq:.3e} T_final {et:.3e} max|dQ| {np.abs(Qg[ok] - ref['Q'][ok]).max():.3e}")
    assert eq < 1e-4 and et < 1e-4
    nc = ws_u32(r.ws, r.debug_views()[5], Qg.shape[0])
    assert np.array_equal(nc[ok], ref["n_contrib"][ok].astype(np.uint32))
    assert np.all(Tg <= 1.0) and np.all(Tg >= 1e-4 * (1 - 1e-5))


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_backward_parity(case, tile):
    if case == "c2" and tile != (16, 16):
        pytest.skip("full-size c2 checked at 16x16")
    g, cams = CASES[case]()
    say(f"[backward] case={case} N={g.n} tile={tile}")
    r, gg, Q, T = _render(g, cams, tile)
    ref = R.render_forward(g, cams)
    w = np.random.default_rng(7).standard_normal(ref["Q"].shape)
    w[ref["margin"] < AMBIGUOUS] = 0.0
    out = r.backward(gg, torch.as_tensor(w, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    w32 = w.astype(np.float32).astype(np.float64)
    og = R.render_backward(g, cams, w32)
    for name in ["means", "log_scales", "quats", "opacity_logits", "queries"]:
        e = rel_err(to_np(getattr(out, name)), og[name])
        say(f"  d_{name}: rel err {e:.3e}")
        assert e < 1e-4, name


def test_tile_shape_invariance_and_determinism():
    g, cams = _scene(1, 5)
    say("[invariance] c1 seed 5")
    outs = []
    for tile in [(16, 16), (8, 8), (16, 8), (32, 8), (8, 32)]:
        _, _, Q, T = _render(g, cams, tile)
        outs.append((to_np(Q), to_np(T)))
    for Qx, Tx in outs[1:]:
        assert np.array_equal(Qx, outs[0][0]) and np.array_equal(Tx, outs[0][1])
    _, _, Q2, _ = _render(g, cams, (16, 16))
    assert np.array_equal(to_np(Q2), outs[0][0])


def test_alpha_at_centre_equals_opacity_gpu():
    cam = scenes.pinhole(80, 60, 70.0)
    g = gaussians([[0.0, 0.0, 2.0]], logits=[logit(0.6)], d=16)
    say("[centre] single Gaussian on axis")
    _, _, Q, T = _render(g, cams_of(cam))
    p = 30 * 80 + 40
    o = np.float32(1.0 / (1.0 + np.exp(-float(g.opacity_logits[0]))))
    np.testing.assert_allclose(to_np(Q)[p], o * g.queries[0], rtol=2e-7)
    assert abs(to_np(T)[p] - (1 - o)) < 1e-7


def test_empty_and_culled_scenes():
    cam = cams_of(scenes.pinhole(37, 29, 30.0))
    say("[edge] all behind the camera")
    g = gaussians([[0.0, 0.0, -1.0], [0.1, 0.0, 0.05]], d=16)
    r, gg, Q, T = _render(g, cam)
    assert np.all(to_np(Q) == 0) and np.all(to_np(T) == 1)
    assert r.counters() == (0, False)
    out = r.backward(gg, torch.ones_like(Q))
    for t in out.tensors():
        assert torch.all(t == 0)
    say("[edge] zero Gaussians")
    g0 = gaussians(np.zeros((0, 3)), d=16)
    ops = _ops()
    r0 = ops.Renderer(cam, 0, 16)
    gg0 = _gpu_gauss(g0)
    Q0, T0 = r0.forward(gg0)
    assert torch.all(Q0 == 0) and torch.all(T0 == 1)


def test_capacity_overflow_is_reported_and_recovered():
    g, cams = _scene(0, 1)
    ops = _ops()
    gg = _gpu_gauss(g)
    say("[capacity] undersized workspace")
    r = ops.Renderer(cams, g.n, 16, capacity=100)
    Q, T = r.forward(gg, check=False)
    need, over = r.counters()
    assert over and need == R.bin_sort(g, cams)["count"]
    Q, T = r.forward(gg)  # grows and re-runs
    assert not r.counters()[1]
    ref = R.render_forward(g, cams)
    ok = ref["margin"] >= AMBIGUOUS
    assert rel_err(to_np(Q)[ok], ref["Q"][ok]) < 1e-4


def test_d32_and_autograd_wrapper():
    sp = scenes.custom_spec("d32", 2000, [scenes.pinhole(50, 40, 40.0)], d=32)
    s = scenes.make_scene(sp, seed=4, with_target=False)
    g = R.Gaussians.of(s)
    say("[autograd] d=32 RenderQueries")
    ops = _ops()
    gg = _gpu_gauss(g)
    for t in gg.tensors():
        t.requires_grad_(True)
    r = ops.Renderer(s.cams, g.n, 32)
    Q, T = ops.RenderQueries.apply(r, *gg.tensors())
    ref = R.render_forward(g, s.cams)
    w = np.random.default_rng(1).standard_normal(ref["Q"].shape)
    w[ref["margin"] < AMBIGUOUS] = 0
    wt = torch.as_tensor(w, dtype=torch.float32, device="cuda")
    (Q * wt).sum().backward()
    og = R.render_backward(g, s.cams, w.astype(np.float32).astype(np.float64))
    for name, t in zip(["means", "log_scales", "quats", "opacity_logits", "queries"], gg.tensors()):
        assert rel_err(to_np(t.grad), og[name]) < 1e-4, name
