"""GPU parity of colour and depth rendering in the query pass (Sec. III-A:
view-independent colour blended by Eq. 2, depth by the same blend of the
centres' camera-space depths) and of the L1 colour/depth loss (Eq. 7-9)
against the FP64 oracles, through the C ABI.

Colour is three more blended channels, so the oracle's reference is its query
blend with the colours as queries (pinned on its own); depth is the oracle's
depth render (pinned by closed forms, the query path and finite
differences).  Bars as for the query map: 1e-4 relative per tensor on pixels
whose oracle walk takes no threshold decision within 1e-5 of a threshold
(upstream gradients zeroed on the others).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import raster as R  # noqa: E402
from oracle import rgbd_loss_oracle as RL  # noqa: E402
from paper_2602_12314_amd import scenes  # noqa: E402
from tests.gpu_helpers import AMBIGUOUS, rel_err, say, to_np  # noqa: E402
from tests.oracle_helpers import cams_of  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _gpu_gauss(g):
    from paper_2602_12314_amd import ops
    return ops.Gaussians(_dev(g.means), _dev(g.log_scales), _dev(g.quats), _dev(g.opacity_logits),
                         _dev(g.queries))


def _multiview(seed=3):
    pose = scenes.look_at_origin((1.2, 0.0, -2.4))
    cams = cams_of(scenes.pinhole(70, 45, 50.0, pose), scenes.pinhole(37, 29, 30.0),
                   scenes.pinhole(64, 64, 60.0, scenes.look_at_origin((-2.0, 0.0, 1.0))))
    sp = scenes.custom_spec("mv", 3000, [scenes.pinhole(37, 29, 30.0)], d=16,
                            box=((-1.5, 1.5), (-1, 1), (-1.5, 1.5)))
    s = scenes.make_scene(sp, seed=seed, with_target=False)
    g = R.Gaussians.of(s)
    g.means[:, 2] += 1.5
    return g, cams


def _scene(i, seed):
    s = scenes.make_scene(scenes.spec(i), seed=seed, with_target=False)
    return R.Gaussians.of(s), s.cams


CASES = {"c0": lambda: _scene(0, 0), "c1": lambda: _scene(1, 1), "multiview_ragged": _multiview,
         "c2_d32": lambda: _scene(2, 2)}


def _colors(n, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (n, 3)).astype(np.float32)


def _with_queries(g, q):
    import copy
    h = copy.copy(g)
    h.queries = np.ascontiguousarray(q, dtype=np.float32)
    return h


@pytest.mark.parametrize("case", list(CASES))
def test_rgbd_forward_parity(case):
    from paper_2602_12314_amd import ops
    g, cams = CASES[case]()
    col = _colors(g.n, 1)
    say(f"[rgbd forward] case={case} N={g.n} d={g.d}")
    r = ops.Renderer(cams, g.n, g.d)
    gg = _gpu_gauss(g)
    Q, rgb, depth, T = r.forward_rgbd(gg, _dev(col))
    Q0, T0 = r.forward(gg)
    torch.cuda.synchronize()
    # the query map and transmittance are untouched by the extra channels
    assert torch.equal(Q, Q0) and torch.equal(T, T0)
    ref = R.render_forward(g, cams)
    refc = R.render_forward(_with_queries(g, col), cams)
    ok = ref["margin"] >= AMBIGUOUS
    ec = rel_err(to_np(rgb)[ok], refc["Q"][ok])
    ez = rel_err(to_np(depth)[ok], ref["Z"][ok])
    say(f"  rel err rgb {ec:.3e} depth {ez:.3e}, ambiguous {(~ok).sum()}")
    assert ec < 1e-4 and ez < 1e-4
    assert (to_np(depth) > 0).sum() > 0.3 * depth.numel()


@pytest.mark.parametrize("case", ["c0", "multiview_ragged", "c1", "c2_d32"])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_rgbd_backward_parity(case, tile):
    from paper_2602_12314_amd import ops
    g, cams = CASES[case]()
    if case in ("c1", "c2_d32") and tile != (16, 16):
        pytest.skip("full-size c1 and c2 checked at 16x16")
    col = _colors(g.n, 2)
    say(f"[rgbd backward] case={case} N={g.n} tile={tile}")
    r = ops.Renderer(cams, g.n, g.d, tile=tile)
    gg = _gpu_gauss(g)
    r.forward_rgbd(gg, _dev(col))
    ref = R.render_forward(g, cams)
    amb = ref["margin"] < AMBIGUOUS
    rng = np.random.default_rng(9)
    w = rng.standard_normal(ref["Q"].shape)
    wc = rng.standard_normal((ref["Q"].shape[0], 3))
    wz = rng.standard_normal(ref["Q"].shape[0])
    for a in (w, wc):
        a[amb] = 0.0
    wz[amb] = 0.0
    w, wc, wz = (a.astype(np.float32) for a in (w, wc, wz))
    out, dcol = r.backward_rgbd(gg, _dev(col), _dev(w), _dev(wc), _dev(wz))
    torch.cuda.synchronize()
    gq = _with_queries(g, np.concatenate([g.queries, col], axis=1))
    og = R.render_backward(gq, cams, np.concatenate([w, wc], axis=1).astype(np.float64), *tile,
                           dZ=wz.astype(np.float64))
    checks = {"means": og["means"], "log_scales": og["log_scales"], "quats": og["quats"],
              "opacity_logits": og["opacity_logits"], "queries": og["queries"][:, :g.d]}
    for name, refv in checks.items():
        e = rel_err(to_np(getattr(out, name)), refv)
        say(f"  d_{name}: rel err {e:.3e}")
        assert e < 1e-4, name
    e = rel_err(to_np(dcol), og["queries"][:, g.d:])
    say(f"  d_colors: rel err {e:.3e}")
    assert e < 1e-4


def test_rgbd_backward_depth_only_reaches_the_means():
    """With only a depth gradient the queries and colours get nothing, and the
    means' gradient matches the oracle's depth adjoint."""
    from paper_2602_12314_amd import ops
    g, cams = CASES["c0"]()
    col = _colors(g.n, 4)
    r = ops.Renderer(cams, g.n, g.d)
    gg = _gpu_gauss(g)
    r.forward_rgbd(gg, _dev(col))
    ref = R.render_forward(g, cams)
    P = ref["Q"].shape[0]
    wz = np.random.default_rng(5).standard_normal(P).astype(np.float32)
    wz[ref["margin"] < AMBIGUOUS] = 0.0
    out, dcol = r.backward_rgbd(gg, _dev(col), torch.zeros((P, g.d), device="cuda"),
                                torch.zeros((P, 3), device="cuda"), _dev(wz))
    og = R.render_backward(g, cams, np.zeros((P, g.d)), dZ=wz.astype(np.float64))
    assert float(to_np(out.queries).__abs__().max()) == 0.0 and float(to_np(dcol).__abs__().max()) == 0.0
    e = rel_err(to_np(out.means), og["means"])
    say(f"[rgbd depth only] d_means rel err {e:.3e}")
    assert e < 1e-4


@pytest.mark.parametrize("n,holes", [(307200, 0.1), (1001, 0.5), (7, 0.0), (300, 1.0), (0, 0.0)])
def test_l1_loss_parity(n, holes):
    from paper_2602_12314_amd import ops
    rng = np.random.default_rng(n + 1)
    rgb, rgb_obs = rng.uniform(0, 1, (n, 3)).astype(np.float32), rng.uniform(0, 1, (n, 3)).astype(np.float32)
    depth, depth_obs = rng.uniform(0.5, 4, n).astype(np.float32), rng.uniform(0.5, 4, n).astype(np.float32)
    depth_obs[rng.uniform(size=n) < holes] = 0.0
    if n > 3:
        rgb[3] = rgb_obs[3]  # ties: zero gradient
        depth[3] = depth_obs[3] = 2.0
    say(f"[rgbd l1] n={n} holes={holes}")
    loss, d_rgb, d_depth = ops.rgbd_l1_loss(_dev(rgb).reshape(n, 3), _dev(rgb_obs).reshape(n, 3), _dev(depth),
                                            _dev(depth_obs), 0.2, 0.1)
    ref = RL.l1_losses(rgb, rgb_obs, depth, depth_obs, 0.2, 0.1)
    assert abs(float(loss) - ref["loss"]) <= 1e-5 * max(abs(ref["loss"]), 1e-30) + 1e-12
    np.testing.assert_allclose(to_np(d_rgb), ref["d_rgb"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(to_np(d_depth), ref["d_depth"], rtol=1e-6, atol=0)


SSIM_VIEWS = {"640x480": [(640, 480)], "ragged_three_views": [(37, 29), (70, 45), (5, 3)]}


@pytest.mark.parametrize("views", list(SSIM_VIEWS))
def test_ssim_parity(views):
    from oracle import ssim_oracle as SS
    from paper_2602_12314_amd import ops
    sizes = SSIM_VIEWS[views]
    cams = cams_of(*[scenes.pinhole(w, h, 50.0) for w, h in sizes])
    P = sum(w * h for w, h in sizes)
    rng = np.random.default_rng(P)
    x = rng.uniform(0, 1, (P, 3)).astype(np.float32)
    y = np.clip(x + 0.15 * rng.standard_normal((P, 3)), 0, 1).astype(np.float32)
    say(f"[ssim] views={views} P={P}")
    loss, d = ops.ssim_loss(_dev(x), _dev(y), cams, 0.8)
    ref = SS.ssim_loss(x, y, sizes)
    rl = 0.8 * ref["loss"]
    say(f"  loss {float(loss):.7f} ref {rl:.7f}; grad rel err {rel_err(to_np(d), 0.8 * ref['d_rgb']):.3e}")
    assert abs(float(loss) - rl) < 1e-5 * max(1.0, abs(rl))
    assert rel_err(to_np(d), 0.8 * ref["d_rgb"]) < 1e-4
    # accumulate: added to what is there
    base = torch.ones((P, 3), device="cuda")
    _, d2 = ops.ssim_loss(_dev(x), _dev(y), cams, 0.8, d_rgb=base)
    np.testing.assert_allclose(to_np(d2), 1.0 + to_np(d), rtol=0, atol=1e-6)


def test_ssim_identical_images():
    from paper_2602_12314_amd import ops
    cams = cams_of(scenes.pinhole(33, 20, 30.0))
    x = np.random.default_rng(1).uniform(0, 1, (33 * 20, 3)).astype(np.float32)
    loss, d = ops.ssim_loss(_dev(x), _dev(x), cams, 1.0)
    assert abs(float(loss)) < 1e-5
    assert float(np.abs(to_np(d)).max()) < 1e-5


def test_rgbd_empty_scene():
    """No Gaussians: colour and depth are zero, the transmittance one, and the
    backward returns empty gradients."""
    from paper_2602_12314_amd import ops
    cams = cams_of(scenes.pinhole(40, 30, 35.0), scenes.pinhole(17, 9, 20.0))
    P = 40 * 30 + 17 * 9
    z = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    g = ops.Gaussians(z(0, 3), z(0, 3), z(0, 4), z(0), z(0, 16))
    r = ops.Renderer(cams, 0, 16)
    Q, rgb, depth, T = r.forward_rgbd(g, z(0, 3))
    torch.cuda.synchronize()
    assert float(Q.abs().max()) == 0 and float(rgb.abs().max()) == 0 and float(depth.abs().max()) == 0
    assert float((T - 1).abs().max()) == 0
    out, dcol = r.backward_rgbd(g, z(0, 3), z(P, 16), z(P, 3), z(P))
    torch.cuda.synchronize()
    assert dcol.shape == (0, 3) and out.means.shape == (0, 3)
