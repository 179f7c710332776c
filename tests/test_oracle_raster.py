"""Pins of the FP64 renderer oracle against facts fixed by the paper and by
geometry: closed forms, a library rotation, rigid-motion invariance, a
textbook sort, a tile-free brute force, and central finite differences.

Passages: Eq. 1-2 (Sec. III-A), Eq. 3-4 (Sec. III-B).  The 3DGS conventions the
paper defers to are listed in the oracle's header.
"""
import copy

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import raster as R
from paper_2602_12314_amd import scenes
from tests.oracle_helpers import cams_of, gaussians, logit, tiny_scene

CAM0 = scenes.pinhole(80, 60, 70.0)  # the 80x60, f=70, c=(40,30) camera


def _pix(cam, x, y):
    return y * cam.width + x


def test_alpha_at_centre_equals_opacity():
    # A single Gaussian on the optical axis lands on pixel (40, 30); there its
    # Gaussian falloff is exp(0) = 1, so alpha equals the opacity (Eq. 2).
    o = 0.6
    g = gaussians([[0.0, 0.0, 2.0]], logits=[logit(o)], d=16)
    out = R.render_forward(g, cams_of(CAM0))
    o64 = 1.0 / (1.0 + np.exp(-float(g.opacity_logits[0])))
    p = _pix(CAM0, 40, 30)
    np.testing.assert_allclose(out["Q"][p], o64 * g.queries[0].astype(np.float64), rtol=0, atol=1e-15)
    assert out["T_final"][p] == pytest.approx(1.0 - o64, abs=1e-15)
    assert out["n_blended"][p] == 1


def test_projection_on_axis_closed_form():
    # Axis-aligned Gaussian at (0, 0, z): the EWA screen covariance is
    # diag((f sx / z)^2, (f sy / z)^2) plus the dilation.
    z, lsx, lsy, lsz = 2.5, -2.0, -2.6, -3.0
    g = gaussians([[0.0, 0.0, z]], log_scales=[[lsx, lsy, lsz]])
    p = R.project(g, cams_of(CAM0))
    sx, sy = np.exp(float(np.float32(lsx))), np.exp(float(np.float32(lsy)))
    a = (70.0 * float(sx) / z) ** 2 + 0.3
    c = (70.0 * float(sy) / z) ** 2 + 0.3
    np.testing.assert_allclose(p["conic"][0], [1 / a, 0.0, 1 / c], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["uv"][0], [40.0, 30.0], rtol=0, atol=0)
    assert abs(a - c) / 2 > np.sqrt(0.1)  # the eigenvalue floor is inactive here
    assert p["radius"][0] == np.ceil(3.0 * np.sqrt(max(a, c)))
    r = int(p["radius"][0])
    assert list(p["rect"][0]) == [40 - r, 40 + r, 30 - r, 30 + r]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_projection_rotated_matches_library_rotation(seed):
    # On the optical axis with an identity camera, J = diag(f/z, f/z) on x, y,
    # so the conic is inv((f/z)^2 Sigma3[:2,:2] + 0.3 I) with Sigma3 = R S^2 R^T.
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((8, 4))
    ls = rng.normal(-2.5, 0.4, (8, 3))
    z = rng.uniform(1.5, 4.0, 8)
    means = np.stack([np.zeros(8), np.zeros(8), z], 1)
    g = gaussians(means, log_scales=ls, quats=q)
    p = R.project(g, cams_of(CAM0))
    for i in range(8):
        qq = g.quats[i].astype(np.float64)
        Rm = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        s = np.exp(g.log_scales[i].astype(np.float64))
        S3 = Rm @ np.diag(s * s) @ Rm.T
        zz = float(g.means[i, 2])
        S2 = (70.0 / zz) ** 2 * S3[:2, :2] + 0.3 * np.eye(2)
        inv = np.linalg.inv(S2)
        np.testing.assert_allclose(p["conic"][i], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-10)


def test_projection_offaxis_uses_jacobian_of_projection():
    # Off axis (clamp inactive), Sigma2 - 0.3 I = J Sigma3 J^T where J is the
    # Jacobian of the oracle's own centre->pixel map, taken here by central FD.
    rng = np.random.default_rng(7)
    means = np.array([[0.4, -0.3, 2.0], [-0.5, 0.2, 1.7], [0.2, 0.35, 2.6]])
    q = rng.standard_normal((3, 4))
    ls = rng.normal(-2.5, 0.3, (3, 3))
    g = gaussians(means, log_scales=ls, quats=q)
    cams = cams_of(CAM0)
    p = R.project(g, cams)
    for i in range(3):
        J = np.zeros((2, 3))
        for k in range(3):
            gp, gm = copy.deepcopy(g), copy.deepcopy(g)
            h = 1e-3
            gp.means[i, k] += h
            gm.means[i, k] -= h
            hh = float(gp.means[i, k]) - float(gm.means[i, k])
            J[:, k] = (R.project(gp, cams)["uv"][i] - R.project(gm, cams)["uv"][i]) / hh
        qq = g.quats[i].astype(np.float64)
        Rm = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        s = np.exp(g.log_scales[i].astype(np.float64))
        S2 = J @ (Rm @ np.diag(s * s) @ Rm.T) @ J.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(S2)
        np.testing.assert_allclose(p["conic"][i], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=2e-5)


def test_pinhole_projection_closed_form():
    # Pinhole model: u - cx = fx * (x / z); points on one ray share a pixel.
    pts = np.array([[0.3, -0.2, 1.5], [0.6, -0.4, 3.0], [0.15, -0.1, 0.75]])
    g = gaussians(pts, log_scales=np.full((3, 3), -4.0))
    p = R.project(g, cams_of(CAM0))
    expect_u = 40.0 + 70.0 * (0.3 / 1.5)
    expect_v = 30.0 + 70.0 * (-0.2 / 1.5)
    for i in range(3):
        x, y, z = (float(v) for v in g.means[i])
        np.testing.assert_allclose(p["uv"][i], [40 + 70 * x / z, 30 + 70 * y / z], rtol=1e-15)
        np.testing.assert_allclose(p["uv"][i], [expect_u, expect_v], rtol=1e-6)


def test_near_plane_and_offscreen_cull():
    g = gaussians([[0.0, 0.0, 0.1], [0.0, 0.0, -1.0], [50.0, 0.0, 2.0], [0.0, 0.0, 2.0]])
    p = R.project(g, cams_of(CAM0))
    assert list(p["vis"]) == [0, 0, 0, 1]


def _random_rigid(seed):
    rng = np.random.default_rng(seed)
    rot = Rotation.from_quat(rng.standard_normal(4))
    t = rng.uniform(-1, 1, 3)
    return rot, t


@pytest.mark.parametrize("seed", [3, 4])
def test_rigid_motion_invariance(seed):
    # Moving the scene and the camera by the same rigid motion leaves every
    # projected quantity unchanged: pins the world->camera handling.
    g, cams = tiny_scene(seed, n=60)
    rot, t = _random_rigid(seed)
    Tg = np.eye(4)
    Tg[:3, :3] = rot.as_matrix()
    Tg[:3, 3] = t
    g2 = copy.deepcopy(g)
    g2.means[:] = (g.means.astype(np.float64) @ rot.as_matrix().T + t).astype(np.float32)
    qs = g.quats.astype(np.float64)
    r2 = rot * Rotation.from_quat(np.stack([qs[:, 1], qs[:, 2], qs[:, 3], qs[:, 0]], 1))
    xyzw = r2.as_quat()
    g2.quats[:] = np.stack([xyzw[:, 3], xyzw[:, 0], xyzw[:, 1], xyzw[:, 2]], 1).astype(np.float32)
    cams2 = cams.copy()
    vm = cams[0, 6:].astype(np.float64).reshape(4, 4) @ np.linalg.inv(Tg)
    cams2[0, 6:] = vm.reshape(-1).astype(np.float32)
    p1, p2 = R.project(g, cams), R.project(g2, cams2)
    both = (p1["vis"] == 1) & (p2["vis"] == 1)
    assert both.sum() >= 0.9 * p1["vis"].sum() > 10
    np.testing.assert_allclose(p2["uv"][both], p1["uv"][both], rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(p2["conic"][both], p1["conic"][both], rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(p2["z"][both], p1["z"][both], rtol=1e-6)


def test_depth_key_bits_order_preserving():
    # Positive float32 values sort like their bit patterns read as uint32.
    rng = np.random.default_rng(0)
    z = np.concatenate([rng.uniform(0.2, 50, 5000), rng.lognormal(0, 3, 5000) + 0.2]).astype(np.float32)
    bits = z.view(np.uint32)
    assert np.array_equal(np.argsort(z, kind="stable"), np.argsort(bits, kind="stable"))


@pytest.mark.parametrize("tw,th", [(16, 16), (8, 8), (16, 4)])
def test_binning_matches_textbook_sort(tw, th):
    s = scenes.make_scene(scenes.spec(0), seed=5, with_target=False)
    g = R.Gaussians.of(s)
    p = R.project(g, s.cams)
    b = R.bin_sort(g, s.cams, tw, th)
    W = int(s.cams[0, 0])
    tx = (W + tw - 1) // tw
    tiles, deps, recs = [], [], []
    for r in np.nonzero(p["vis"])[0]:
        x0, x1, y0, y1 = p["rect"][r]
        for ty in range(y0 // th, y1 // th + 1):
            for t in range(x0 // tw, x1 // tw + 1):
                tiles.append(ty * tx + t)
                deps.append(p["depth_key"][r])
                recs.append(r)
    tiles, deps, recs = (np.array(a, np.int64) for a in (tiles, deps, recs))
    order = np.lexsort((recs, deps, tiles))
    assert b["count"] == len(tiles)
    assert np.array_equal(b["tiles"], tiles[order])
    assert np.array_equal(b["recs"], recs[order])
    assert np.array_equal(b["depths"], deps[order])
    nt = R.num_tiles(s.cams, tw, th)
    st = np.searchsorted(tiles[order], np.arange(nt), "left")
    en = np.searchsorted(tiles[order], np.arange(nt), "right")
    empty = st == en
    assert np.array_equal(b["ranges"][~empty, 0], st[~empty])
    assert np.array_equal(b["ranges"][~empty, 1], en[~empty])
    assert np.all(b["ranges"][empty] == 0)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (4, 4), (16, 4)])
def test_bruteforce_equals_tile_binned(seed, tile):
    # Tile binning only accelerates the per-pixel definition: same Gaussians in
    # the same order, so the FP64 results are bitwise equal for any tile shape.
    g, cams = tiny_scene(seed, n=50, w=32, h=32, f=28.0)
    bf = R.render_bruteforce(g, cams)
    tb = R.render_forward(g, cams, *tile)
    assert np.array_equal(bf["Q"], tb["Q"])
    assert np.array_equal(bf["T_final"], tb["T_final"])
    assert np.array_equal(bf["n_blended"], tb["n_blended"])


def test_bruteforce_multiview_rotated():
    pose = scenes.look_at_origin((1.5, 0.0, -2.0))
    c1 = scenes.pinhole(33, 21, 25.0, pose)
    c2 = scenes.pinhole(20, 30, 22.0)
    g, _ = tiny_scene(9, n=80, w=33, h=21)
    g.means[:, 2] += 0.5
    cams = cams_of(c1, c2)
    bf = R.render_bruteforce(g, cams)
    tb = R.render_forward(g, cams, 8, 8)
    assert np.array_equal(bf["Q"], tb["Q"])
    assert (bf["n_blended"] > 0).sum() > 100


def _on_axis(zs, opac, qs):
    return gaussians([[0.0, 0.0, z] for z in zs], log_scales=np.full((len(zs), 3), -4.0),
                     logits=[logit(o) for o in opac], queries=qs)


def test_two_gaussians_closed_form():
    q1, q2 = np.array([1.0, 2.0, -1.0, 0.5]), np.array([-0.5, 0.25, 3.0, 1.0])
    o1, o2 = 0.3, 0.7
    cams = cams_of(CAM0)
    p = _pix(CAM0, 40, 30)
    for order in ([1.5, 2.5], [2.5, 1.5]):
        qs = [q1, q2] if order[0] < order[1] else [q2, q1]
        ops = [o1, o2] if order[0] < order[1] else [o2, o1]
        g = _on_axis(order, ops, qs)
        out = R.render_forward(g, cams)
        a1 = 1 / (1 + np.exp(-float(np.float32(logit(o1)))))
        a2 = 1 / (1 + np.exp(-float(np.float32(logit(o2)))))
        ref = a1 * np.float32(q1).astype(np.float64) + (1 - a1) * a2 * np.float32(q2).astype(np.float64)
        np.testing.assert_allclose(out["Q"][p], ref, rtol=1e-14)
        assert out["T_final"][p] == pytest.approx((1 - a1) * (1 - a2), rel=1e-14)


def test_equal_depth_ties_follow_index():
    q1, q2 = np.array([1.0, 0.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0, 0.0])
    g = _on_axis([2.0, 2.0], [0.5, 0.5], [q1, q2])
    out = R.render_forward(g, cams_of(CAM0))
    a = 1 / (1 + np.exp(-float(np.float32(logit(0.5)))))
    np.testing.assert_allclose(out["Q"][_pix(CAM0, 40, 30)], [a, (1 - a) * a, 0, 0], rtol=1e-14)


def test_termination_before_transmittance_floor():
    # alpha = 0.95 each: T = 0.05, 0.0025, 1.25e-4, then 6.25e-6 < 1e-4 stops.
    n = 6
    g = _on_axis([1.0 + 0.2 * k for k in range(n)], [0.95] * n, np.eye(n)[:, :4])
    out = R.render_forward(g, cams_of(CAM0))
    p = _pix(CAM0, 40, 30)
    a = 1 / (1 + np.exp(-float(np.float32(logit(0.95)))))
    assert out["n_blended"][p] == 3
    assert out["T_final"][p] == pytest.approx((1 - a) ** 3, rel=1e-14)


def test_alpha_clamp_and_skip():
    # opacity above the clamp blends with alpha = 0.99; below 1/255 is skipped.
    g = _on_axis([2.0], [0.999], [np.ones(4)])
    out = R.render_forward(g, cams_of(CAM0))
    p = _pix(CAM0, 40, 30)
    assert out["T_final"][p] == pytest.approx(0.01, rel=1e-15)
    g = _on_axis([2.0], [0.003], [np.ones(4)])
    out = R.render_forward(g, cams_of(CAM0))
    assert out["T_final"][p] == 1.0 and np.all(out["Q"][p] == 0)


def test_transmittance_bounds_config0():
    s = scenes.make_scene(scenes.spec(0), seed=0, with_target=False)
    out = R.render_forward(R.Gaussians.of(s), s.cams)
    T = out["T_final"]
    assert np.all(T <= 1.0) and np.all(T >= 1e-4)
    # more blended Gaussians never raise the transmittance
    order = np.argsort(out["n_blended"], kind="stable")
    assert np.all(T[out["n_blended"] == 0] == 1.0)
    assert T[order][-1] <= T[order][0]


def _fd_check(g, cams, seed, hrel=1e-5, tol=2e-6, tile=(16, 16), depth=False):
    f = R.render_forward(g, cams, *tile)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(f["Q"].shape)
    wz = rng.standard_normal(f["Z"].shape) if depth else np.zeros(f["Z"].shape)
    gr = R.render_backward(g, cams, w, *tile, dZ=wz if depth else None)
    checked = 0
    for name in ["means", "log_scales", "quats", "opacity_logits", "queries"]:
        arr = getattr(g, name)
        errs, mags = [], []
        for idx in np.ndindex(arr.shape):
            x0 = float(arr[idx])
            h = hrel * max(1.0, abs(x0))
            gp, gm = copy.deepcopy(g), copy.deepcopy(g)
            getattr(gp, name)[idx] = np.float32(x0 + h)
            getattr(gm, name)[idx] = np.float32(x0 - h)
            hp = float(getattr(gp, name)[idx]) - x0
            hm = x0 - float(getattr(gm, name)[idx])
            op, om = R.render_forward(gp, cams, *tile), R.render_forward(gm, cams, *tile)
            if not (np.array_equal(op["hash"], f["hash"]) and np.array_equal(om["hash"], f["hash"])):
                continue  # a decision flipped inside the stencil: not differentiable there
            fd = (((op["Q"] * w).sum() + (op["Z"] * wz).sum()) -
                  ((om["Q"] * w).sum() + (om["Z"] * wz).sum())) / (hp + hm)
            errs.append(abs(fd - gr[name][idx]))
            mags.append(abs(gr[name][idx]))
        errs, mags = np.array(errs), np.array(mags)
        assert len(errs) > 0.8 * arr.size, name
        assert errs.max() <= tol * max(mags.max(), 1e-12), (name, errs.max(), mags.max())
        checked += len(errs)
    return checked


def test_fd_gradients_identity_camera():
    g, cams = tiny_scene(3, n=30)
    assert _fd_check(g, cams, 2) > 300


def test_fd_gradients_rotated_two_views():
    pose = scenes.look_at_origin((1.0, 0.0, -2.5))
    g, _ = tiny_scene(11, n=25)
    g.means[:, 2] -= 1.0
    cams = cams_of(scenes.pinhole(30, 24, 24.0, pose), scenes.pinhole(26, 20, 20.0))
    assert _fd_check(g, cams, 4, tile=(8, 8)) > 250


def test_fd_gradients_with_fov_clamp_active():
    # Wide spread and a narrow camera: many centres lie beyond 1.3 tan(fov/2)
    # while their footprint still reaches the image.
    rng = np.random.default_rng(5)
    means = np.stack([rng.uniform(-1.6, 1.6, 30), rng.uniform(-0.3, 0.3, 30), rng.uniform(1.0, 1.6, 30)], 1)
    g = gaussians(means, log_scales=rng.normal(-1.2, 0.2, (30, 3)), quats=rng.standard_normal((30, 4)),
                  logits=rng.normal(-1.0, 0.5, 30), d=3, seed=5)
    cams = cams_of(scenes.pinhole(24, 16, 40.0))
    p = R.project(g, cams)
    lim = 1.3 * 24 / (2 * 40.0)
    rx = p["z"] * 0 + (g.means[:, 0] / g.means[:, 2])
    assert np.sum((np.abs(rx) > lim) & (p["vis"] == 1)) >= 3
    _fd_check(g, cams, 6, tol=5e-6)


# ---------------------------------------------------------------- depth render

def test_depth_at_centre_and_two_gaussians_closed_form():
    # Sec. III-A: depth is blended with the weights of Eq. 2.  On the axis the
    # centre pixel sees alpha = opacity, so one Gaussian gives o z and two give
    # a1 z1 + (1 - a1) a2 z2.
    cams = cams_of(CAM0)
    p = _pix(CAM0, 40, 30)
    g = _on_axis([2.0], [0.6], [np.ones(4)])
    out = R.render_forward(g, cams)
    o = 1 / (1 + np.exp(-float(np.float32(logit(0.6)))))
    assert out["Z"][p] == pytest.approx(o * 2.0, rel=1e-14)
    g = _on_axis([1.5, 2.5], [0.3, 0.7], [np.ones(4), np.ones(4)])
    out = R.render_forward(g, cams)
    a1 = 1 / (1 + np.exp(-float(np.float32(logit(0.3)))))
    a2 = 1 / (1 + np.exp(-float(np.float32(logit(0.7)))))
    assert out["Z"][p] == pytest.approx(a1 * 1.5 + (1 - a1) * a2 * 2.5, rel=1e-14)


def test_depth_is_the_query_blend_of_the_centre_depths():
    # With each Gaussian's query set to its camera-space depth (one camera), the
    # pinned query blend must reproduce the depth render.
    g, cams = tiny_scene(4, n=60, w=32, h=32, f=28.0)
    z = R.project(g, cams)["z"]
    gz = copy.deepcopy(g)
    gz.queries = np.ascontiguousarray(z[:, None].astype(np.float32))
    out = R.render_forward(g, cams)
    ref = R.render_forward(gz, cams)
    np.testing.assert_allclose(out["Z"], ref["Q"][:, 0], rtol=1e-6, atol=1e-12)
    assert (out["Z"] > 0).sum() > 200


def test_bruteforce_depth_equals_tile_binned():
    g, cams = tiny_scene(2, n=50, w=32, h=32, f=28.0)
    bf = R.render_bruteforce(g, cams)
    tb = R.render_forward(g, cams, 8, 8)
    assert np.array_equal(bf["Z"], tb["Z"])


def test_fd_gradients_with_depth_identity_camera():
    g, cams = tiny_scene(3, n=30)
    assert _fd_check(g, cams, 7, depth=True) > 300


def test_fd_gradients_with_depth_rotated_two_views():
    pose = scenes.look_at_origin((1.0, 0.0, -2.5))
    g, _ = tiny_scene(11, n=25)
    g.means[:, 2] -= 1.0
    cams = cams_of(scenes.pinhole(30, 24, 24.0, pose), scenes.pinhole(26, 20, 20.0))
    assert _fd_check(g, cams, 8, tile=(8, 8), depth=True) > 250


# ------------------------------------------------ footprint and walk properties

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_footprint_rect_is_the_pixel_set_at_non_integer_centres(seed):
    # The footprint of a record is exactly {px : |px - u| <= r} x {py : |py - v| <= r}
    # intersected with the image, enumerated here pixel by pixel from the
    # projected (u, v, r).  Off-axis centres are non-integer, so a ceil/floor
    # slip at either end of the interval shows up.
    pose = scenes.look_at_origin((0.7, -0.2, -2.6))
    g, _ = tiny_scene(seed, n=400, w=61, h=47, f=40.0)
    g.means[:, 2] += 0.4
    cams = cams_of(scenes.pinhole(61, 47, 40.0), scenes.pinhole(45, 38, 33.0, pose))
    p = R.project(g, cams)
    checked = 0
    for r in np.nonzero(p["vis"])[0]:
        c = r // g.n
        W, H = int(cams[c, 0]), int(cams[c, 1])
        u, v = p["uv"][r]
        rad = p["radius"][r]
        xs = np.arange(W)
        ys = np.arange(H)
        inx = xs[np.abs(xs - u) <= rad]
        iny = ys[np.abs(ys - v) <= rad]
        assert len(inx) and len(iny)
        assert list(p["rect"][r]) == [inx.min(), inx.max(), iny.min(), iny.max()], (r, u, v, rad)
        checked += u != np.floor(u)
    assert checked > 300
    # and no record outside the image survives
    for r in np.nonzero(p["vis"] == 0)[0]:
        c = r // g.n
        if p["z"][r] <= 0.2 or p["radius"][r] == 0:
            continue
        W, H = int(cams[c, 0]), int(cams[c, 1])
        u, v = p["uv"][r]
        rad = p["radius"][r]
        assert not ((np.abs(np.arange(W) - u) <= rad).any() and (np.abs(np.arange(H) - v) <= rad).any())


def test_transmittance_non_increasing_along_every_walk():
    # Along each pixel's walk T_0 = 1, T_{k+1} = T_k (1 - alpha_k) <= T_k, every
    # alpha in [1/255, 0.99], every T in [1e-4, 1], and T_final the product.
    s = scenes.make_scene(scenes.spec(0), seed=3, with_target=False)
    g = R.Gaussians.of(s)
    P = R.n_pixels(s.cams)
    pix = np.arange(P)
    wk = R.pixel_walks(g, s.cams, pix, max_len=1024)
    f = R.render_forward(g, s.cams)
    assert np.array_equal(wk["count"], f["n_blended"])
    assert np.array_equal(wk["T_final"], f["T_final"])
    assert wk["count"].max() < 1024 and wk["count"].sum() > 10 * P
    for i in range(P):
        k = wk["count"][i]
        if k == 0:
            assert wk["T_final"][i] == 1.0
            continue
        a = wk["alpha"][i, :k]
        T = wk["T_before"][i, :k]
        assert T[0] == 1.0
        assert np.all(a >= 1.0 / 255.0) and np.all(a <= 0.99)
        assert np.all(np.diff(T) <= 0.0)
        np.testing.assert_array_equal(T[1:], T[:-1] * (1.0 - a[:-1]))
        assert wk["T_final"][i] == T[-1] * (1.0 - a[-1])
        assert wk["T_final"][i] >= 1e-4 and wk["T_final"][i] <= T[-1]
        np.testing.assert_allclose(wk["T_final"][i], np.prod(1.0 - a), rtol=1e-12)


def test_exp_cw_within_one_ulp_of_exp():
    # The float32 exp of the projection (Cody-Waite reduction and a degree-7
    # Taylor polynomial) against the FP64 exp, over the range log-scales and
    # opacity logits take and beyond: within one float32 ulp, exact at 0.
    rng = np.random.default_rng(5)
    x = np.concatenate([np.linspace(-30.0, 20.0, 200001, dtype=np.float32),
                        rng.uniform(-87.0, 88.0, 100000).astype(np.float32)])
    y = R.exp_cw(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(y - ref) / ulp) <= 1.0
    assert R.exp_cw(np.zeros(1))[0] == 1.0


@pytest.mark.parametrize("idx", [1, 2, 4])
def test_float32_decisions_match_fp64_away_from_thresholds(idx):
    # The integer decisions of the projection (culling, radius, footprint,
    # depth key) are taken in float32, the precision of the projection they
    # belong to.  Taken again in FP64 they must agree wherever FP64 puts them
    # farther from a threshold than float32 rounding can move them (1e-3 px,
    # or 1e-3 of depth at the near plane), and the float32 depth z must lie
    # within the rounding bound of a four-term float32 sum, 4 u (|w0 mx| +
    # |w1 my| + |w2 mz| + |t|), of the FP64 z.
    sp = scenes.spec(idx)
    s = scenes.make_scene(sp, seed=0, with_target=False)
    g = R.Gaussians.of(s)
    p32 = R.project(g, s.cams)
    p64 = R.project_decisions64(g, s.cams)
    v32, v64 = p32["vis"] == 1, p64["vis"] == 1
    safe = p64["margin"] > 1e-3
    assert np.array_equal(v32[safe], v64[safe])
    both = v32 & v64
    differ = both & np.any(p32["rect"] != p64["rect"], axis=1)
    assert not np.any(differ & safe)
    n_flip = int(np.count_nonzero((v32 != v64) | differ))
    print(f"[decisions] {sp.name}: {int(v32.sum())} visible, {n_flip} records with another rect or "
          f"visibility in FP64 (all within {p64['margin'][(v32 != v64) | differ].max(initial=0.0):.2e} px "
          f"of a threshold)")
    assert n_flip <= 1e-3 * max(int(v32.sum()), 1)
    cams = np.asarray(s.cams, np.float64)
    n = g.n
    z32 = p32["depth_key"][both].view(np.float32).astype(np.float64)
    rec = np.nonzero(both)[0]
    c, i = rec // n, rec % n
    vm = cams[c, 6:22].reshape(-1, 4, 4)
    m = g.means.astype(np.float64)[i]
    terms = np.abs(vm[:, 2, :3] * m).sum(1) + np.abs(vm[:, 2, 3])
    u = 2.0 ** -24
    assert np.all(np.abs(z32 - p32["z"][both]) <= 4 * u / (1 - 4 * u) * terms)
