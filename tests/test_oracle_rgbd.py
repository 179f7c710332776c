"""Pins of the FP64 L1 colour/depth loss oracle (Eq. 7-9): torch's L1 loss and
its autograd, closed forms, finite differences away from ties."""
import numpy as np
import pytest

from oracle import rgbd_loss_oracle as RL

torch = pytest.importorskip("torch")


def _inputs(seed, n=50, holes=0.2):
    rng = np.random.default_rng(seed)
    rgb, rgb_obs = rng.uniform(0, 1, (n, 3)), rng.uniform(0, 1, (n, 3))
    depth = rng.uniform(0.5, 4.0, n)
    depth_obs = rng.uniform(0.5, 4.0, n)
    depth_obs[rng.uniform(size=n) < holes] = 0.0
    return rgb, rgb_obs, depth, depth_obs


def test_matches_torch_l1_and_autograd():
    rgb, rgb_obs, depth, depth_obs = _inputs(0)
    r = RL.l1_losses(rgb, rgb_obs, depth, depth_obs, 0.2, 0.1)
    tr = torch.tensor(rgb, requires_grad=True)
    tz = torch.tensor(depth, requires_grad=True)
    valid = torch.tensor(depth_obs > 0)
    L = 0.2 * torch.nn.functional.l1_loss(tr, torch.tensor(rgb_obs)) + \
        0.1 * torch.nn.functional.l1_loss(tz[valid], torch.tensor(depth_obs)[valid])
    L.backward()
    assert abs(L.item() - r["loss"]) < 1e-14
    np.testing.assert_allclose(r["d_rgb"], tr.grad.numpy(), rtol=1e-14)
    np.testing.assert_allclose(r["d_depth"], tz.grad.numpy(), rtol=1e-14, atol=1e-18)


def test_closed_form_and_holes():
    rgb = np.array([[1.0, 0.0, 0.5], [0.2, 0.2, 0.2]])
    obs = np.array([[0.5, 0.5, 0.5], [0.2, 0.4, 0.0]])
    depth = np.array([2.0, 3.0])
    dobs = np.array([1.5, 0.0])  # the second pixel has no measurement
    r = RL.l1_losses(rgb, obs, depth, dobs, 1.0, 1.0)
    assert r["rgb_term"] == pytest.approx((0.5 + 0.5 + 0 + 0 + 0.2 + 0.2) / 6)
    assert r["depth_term"] == pytest.approx(0.5)
    assert r["n_valid"] == 1
    np.testing.assert_array_equal(r["d_depth"], [1.0, 0.0])
    np.testing.assert_array_equal(r["d_rgb"][0], [1 / 6, -1 / 6, 0.0])  # zero at the tie
    r0 = RL.l1_losses(rgb, obs, depth, np.zeros(2), 1.0, 1.0)
    assert r0["depth_term"] == 0.0 and np.all(r0["d_depth"] == 0.0)


def test_finite_differences():
    rgb, rgb_obs, depth, depth_obs = _inputs(3, n=20, holes=0.3)
    r = RL.l1_losses(rgb, rgb_obs, depth, depth_obs, 0.7, 0.3)
    h = 1e-7
    for arr, grad in ((rgb, r["d_rgb"]), (depth, r["d_depth"])):
        for idx in list(np.ndindex(arr.shape))[:25]:
            p, m = arr.copy(), arr.copy()
            p[idx] += h
            m[idx] -= h
            args_p = (p, rgb_obs, depth, depth_obs) if arr is rgb else (rgb, rgb_obs, p, depth_obs)
            args_m = (m, rgb_obs, depth, depth_obs) if arr is rgb else (rgb, rgb_obs, m, depth_obs)
            fd = (RL.l1_losses(*args_p, 0.7, 0.3)["loss"] - RL.l1_losses(*args_m, 0.7, 0.3)["loss"]) / (2 * h)
            assert abs(fd - grad[idx]) < 1e-6
