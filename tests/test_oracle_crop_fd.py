"""Central finite differences of the FP64 oracle on the 64-pixel crop of the
1200x680 workload (300k Gaussians, d = 32, M = 512, D = 768): the gradient of
the crop's feature loss (Eq. 6 over the crop pixels, decode of Eq. 5, query
map of Eq. 4 / Eq. 2) with respect to every parameter of every Gaussian whose
footprint overlaps the crop, and to seeded entries of Q, K and V.  At these
list lengths (about 140 footprint hits and 85 blends per pixel) the adjoint of
the compositing and of the attention are exercised as the full-size workload
uses them, which the tiny-scene pins do not.

The crop is the 8 x 8 window [596, 604) x [336, 344).  Only Gaussians whose
footprint overlaps it can reach its pixels (the per-pixel footprint test), so
the sub-scene of those Gaussians, kept in their original order, renders the
crop exactly like the whole scene; a test below checks that bitwise.
"""
import numpy as np
import pytest

from oracle import decode_oracle as DO
from oracle import raster as R
from paper_2602_12314_amd import scenes

X0, Y0, CW, CH = 596, 336, 8, 8
LAMBDA = 0.1
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "queries")


@pytest.fixture(scope="module")
def crop():
    sp = scenes.spec(2)
    s = scenes.make_scene(sp, seed=0, with_target=False)
    g = R.Gaussians.of(s)
    p = R.project(g, s.cams)
    rect = p["rect"]
    ov = (p["vis"] == 1) & (rect[:, 0] <= X0 + CW - 1) & (rect[:, 1] >= X0) & \
         (rect[:, 2] <= Y0 + CH - 1) & (rect[:, 3] >= Y0)
    idx = np.nonzero(ov)[0]
    sub = R.Gaussians(*[np.ascontiguousarray(getattr(g, k)[idx]) for k in GROUPS])
    cam = s.cams[0]
    # target rows of the crop by the workload's recipe (32 unit prototypes in
    # R^768 on a Voronoi partition of the image, N(0, 0.05^2) noise, renormalised)
    rng = np.random.default_rng(20)
    protos = rng.standard_normal((sp.n_sites, sp.D))
    protos /= np.linalg.norm(protos, axis=1, keepdims=True)
    sites = rng.uniform(0, 1, (sp.n_sites, 2)) * np.array([1200.0, 680.0])
    ys, xs = np.mgrid[Y0:Y0 + CH, X0:X0 + CW]
    pix = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float64)
    lab = ((pix[:, None, :] - sites[None]) ** 2).sum(-1).argmin(1)
    T = protos[lab] + sp.noise * rng.standard_normal((CW * CH, sp.D))
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    K = s.K.astype(np.float64)
    K0 = K + 0.01 * rng.standard_normal(K.shape)  # a trust-region gradient that is not zero
    return dict(s=s, g=g, idx=idx, sub=sub, cam=cam, T=T, K=K, V=s.V.astype(np.float64), K0=K0)


def _crop_pixels():
    ys, xs = np.mgrid[Y0:Y0 + CH, X0:X0 + CW]
    return (ys * 1200 + xs).ravel()


def test_crop_subscene_renders_like_the_whole_scene(crop):
    # the restriction to overlapping Gaussians changes nothing inside the crop,
    # and the window function equals the tile-binned full-frame render there
    w_sub = R.render_window(crop["sub"], crop["cam"], X0, Y0, CW, CH)
    w_all = R.render_window(crop["g"], crop["cam"], X0, Y0, CW, CH)
    f_sub = R.render_forward(crop["sub"], crop["s"].cams)
    assert np.array_equal(w_sub["Q"], w_all["Q"])
    assert np.array_equal(w_sub["T_final"], w_all["T_final"])
    assert np.array_equal(f_sub["Q"][_crop_pixels()], w_sub["Q"])
    # realistic list lengths: every crop pixel is hit by many Gaussians
    assert f_sub["n_pairs"][_crop_pixels()].min() >= 50
    assert f_sub["n_blended"][_crop_pixels()].mean() >= 40


def _adjoint(crop, gQ):
    dQ = np.zeros((R.n_pixels(crop["s"].cams), crop["sub"].d))
    dQ[_crop_pixels()] = gQ
    return R.render_backward(crop["sub"], crop["s"].cams, dQ)


def _probe_value(gr, name, i, k):
    a, b = R.PARAM_SLICES.get(name, (11, None))
    return gr[name][i, k - a] if gr[name].ndim == 2 else gr[name][i]


def test_crop_fd_every_gaussian_parameter(crop):
    """Central differences of the crop loss, linearised at the point through
    its exact upstream gradient dL/dQ (the chain rule), for every parameter of
    every overlapping Gaussian, against the oracle's compositing adjoint."""
    sub, d = crop["sub"], crop["sub"].d
    Q = R.render_window(sub, crop["cam"], X0, Y0, CW, CH)["Q"]
    ref = DO.loss_and_grads(Q, crop["K"], crop["V"], crop["T"], crop["K0"], LAMBDA)
    gQ = ref["dQ"]
    gr = _adjoint(crop, gQ)
    n = sub.n
    assert n <= 2000  # every overlapping Gaussian is probed (no sampling needed)
    P = 11 + d
    pg = np.repeat(np.arange(n), P)
    pk = np.tile(np.arange(P), n)
    fd, ok = R.fd_window(sub, crop["cam"], X0, Y0, CW, CH, gQ, pg, pk, hrel=1e-5)
    assert ok.mean() > 0.99
    adj = np.concatenate([gr["means"], gr["log_scales"], gr["quats"], gr["opacity_logits"][:, None],
                          gr["queries"]], 1).reshape(-1)
    for name, (a, b) in list(R.PARAM_SLICES.items()) + [("queries", (11, P))]:
        sel = ok & (pk >= a) & (pk < b)
        err = np.abs(fd[sel] - adj[sel])
        scale = np.abs(adj[(pk >= a) & (pk < b)]).max()
        assert scale > 0, name
        # truncation O(h^2) and FP64 rounding: well below 1e-6 of the group's largest entry
        assert err.max() <= 1e-6 * scale, (name, err.max(), scale)
    # the probes cover every (Gaussian, parameter) pair of the crop
    assert len(fd) == n * P and n > 500


def test_crop_fd_composed_loss_subset(crop):
    """The full crop loss (render the window, decode, cosine + trust region)
    differenced directly for a seeded subset of Gaussian parameters: the
    composition of the two adjoints is the gradient of the composed loss."""
    sub = crop["sub"]
    Q = R.render_window(sub, crop["cam"], X0, Y0, CW, CH)["Q"]
    base = R.render_window(sub, crop["cam"], X0, Y0, CW, CH)
    ref = DO.loss_and_grads(Q, crop["K"], crop["V"], crop["T"], crop["K0"], LAMBDA)
    gr = _adjoint(crop, ref["dQ"])
    rng = np.random.default_rng(21)
    names = ["means", "log_scales", "quats", "opacity_logits", "queries"]
    checked = 0
    for name in names:
        arr = getattr(sub, name)
        errs, mags = [], []
        for _ in range(12):
            idx = tuple(int(rng.integers(0, m)) for m in arr.shape)
            x0 = float(arr[idx])
            h = 1e-5 * max(1.0, abs(x0))
            vals, steps, same = [], [], True
            for sgn in (1.0, -1.0):
                arr[idx] = np.float32(x0 + sgn * h)
                steps.append(abs(float(arr[idx]) - x0))
                wv = R.render_window(sub, crop["cam"], X0, Y0, CW, CH)
                same &= np.array_equal(wv["hash"], base["hash"])
                vals.append(DO.feature_loss(wv["Q"], crop["K"], crop["V"], crop["T"], crop["K0"], LAMBDA))
            arr[idx] = np.float32(x0)
            if not same:
                continue
            fd = (vals[0] - vals[1]) / (steps[0] + steps[1])
            an = gr[name][idx]
            errs.append(abs(fd - an))
            mags.append(abs(an))
        assert len(errs) >= 10, name
        scale = max(np.abs(gr[name]).max(), 1e-300)
        assert max(errs) <= 2e-6 * scale, (name, max(errs), scale)
        checked += len(errs)
    assert checked >= 50


def test_crop_fd_dictionary_and_queries(crop):
    """Central differences of the crop loss in 200 seeded entries each of K
    and V and 256 of the query map Q against the oracle's dK, dV, dQ
    (dK includes the trust-region term 2 lambda (K - K0))."""
    sub = crop["sub"]
    Q = R.render_window(sub, crop["cam"], X0, Y0, CW, CH)["Q"]
    K, V, T, K0 = crop["K"].copy(), crop["V"].copy(), crop["T"], crop["K0"]
    ref = DO.loss_and_grads(Q, K, V, T, K0, LAMBDA)
    rng = np.random.default_rng(22)
    for name, arr, an, count in (("K", K, ref["dK"], 200), ("V", V, ref["dV"], 200), ("Q", Q, ref["dQ"], 256)):
        flat = rng.choice(arr.size, count, replace=False)
        errs = []
        for f in flat:
            idx = np.unravel_index(f, arr.shape)
            x0 = arr[idx]
            h = 1e-6 * max(1.0, abs(x0))
            arr[idx] = x0 + h
            lp = DO.feature_loss(Q, K, V, T, K0, LAMBDA)
            arr[idx] = x0 - h
            lm = DO.feature_loss(Q, K, V, T, K0, LAMBDA)
            arr[idx] = x0
            errs.append(abs((lp - lm) / (2 * h) - an[idx]))
        scale = np.abs(an).max()
        assert max(errs) <= 1e-6 * scale, (name, max(errs), scale)
