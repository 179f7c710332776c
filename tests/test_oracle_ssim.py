"""Pins of the FP64 SSIM oracle (Eq. 7): identity, symmetry, the closed form on
constant images, torch's conv2d with autograd as an independent formulation,
and finite differences."""
import numpy as np
import pytest

from oracle import ssim_oracle as SS

torch = pytest.importorskip("torch")


def _img(seed, h, w):
    return np.random.default_rng(seed).uniform(0, 1, (h * w, 3))


def test_identical_images_have_ssim_one():
    x = _img(0, 20, 30)
    r = SS.ssim_loss(x, x, [(30, 20)])
    assert abs(r["loss"]) < 1e-12
    np.testing.assert_allclose(r["d_rgb"], 0.0, atol=1e-12)


def test_symmetric_in_its_arguments():
    x, y = _img(1, 17, 23), _img(2, 17, 23)
    assert SS.ssim_loss(x, y, [(23, 17)])["loss"] == pytest.approx(SS.ssim_loss(y, x, [(23, 17)])["loss"], rel=1e-13)


def test_constant_images_interior_closed_form():
    # away from the border the window sums to 1: mu = the constant, sigma = 0,
    # S = (2 a b + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    h, w = 31, 31
    x = np.full((h * w, 3), a)
    y = np.full((h * w, 3), b)
    S, _ = SS.ssim_view(x.reshape(h, w, 3), y.reshape(h, w, 3))
    ref = (2 * a * b + SS.C1) * SS.C2 / ((a * a + b * b + SS.C1) * SS.C2)
    np.testing.assert_allclose(S[5:-5, 5:-5], ref, rtol=1e-11)  # the window sums to 1 up to rounding


def _torch_ssim_loss(x, y, sizes):
    import torch.nn.functional as F
    win = torch.tensor(SS.window())[None, None].repeat(3, 1, 1, 1)
    tot, off, acc = 0, 0, 0.0
    for w, h in sizes:
        xi = x[off:off + w * h].reshape(h, w, 3).permute(2, 0, 1)[None]
        yi = y[off:off + w * h].reshape(h, w, 3).permute(2, 0, 1)[None]
        f = lambda t: F.conv2d(t, win, padding=5, groups=3)
        mx, my = f(xi), f(yi)
        sxx = f(xi * xi) - mx ** 2
        syy = f(yi * yi) - my ** 2
        sxy = f(xi * yi) - mx * my
        S = (2 * mx * my + SS.C1) * (2 * sxy + SS.C2) / ((mx ** 2 + my ** 2 + SS.C1) * (sxx + syy + SS.C2))
        acc = acc + S.sum()
        tot += 3 * w * h
        off += w * h
    return 1 - acc / tot


def test_matches_torch_conv2d_and_autograd_two_views():
    sizes = [(23, 17), (12, 9)]
    P = sum(w * h for w, h in sizes)
    x, y = _img(3, 1, P), _img(4, 1, P)
    r = SS.ssim_loss(x, y, sizes)
    tx = torch.tensor(x, requires_grad=True)
    L = _torch_ssim_loss(tx, torch.tensor(y), sizes)
    L.backward()
    assert abs(L.item() - r["loss"]) < 1e-13
    np.testing.assert_allclose(r["d_rgb"], tx.grad.numpy(), rtol=1e-9, atol=1e-15)


def test_finite_differences():
    sizes = [(9, 8)]
    x, y = _img(5, 8, 9), _img(6, 8, 9)
    r = SS.ssim_loss(x, y, sizes)
    h = 1e-6
    rng = np.random.default_rng(7)
    for _ in range(20):
        idx = (int(rng.integers(0, x.shape[0])), int(rng.integers(0, 3)))
        p, m = x.copy(), x.copy()
        p[idx] += h
        m[idx] -= h
        fd = (SS.ssim_loss(p, y, sizes)["loss"] - SS.ssim_loss(m, y, sizes)["loss"]) / (2 * h)
        assert abs(fd - r["d_rgb"][idx]) < 1e-8 + 1e-6 * abs(fd)
