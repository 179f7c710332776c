"""Pins of the FP64 decode / loss oracle (Eq. 5-6, Sec. III-B).

- library routine: softmax(Q K^T / sqrt(d)) V is scaled dot-product attention;
  torch's CPU implementation in float64 (forward and autograd) must agree;
- closed forms: a one-hot attention row returns exactly that row of V; Q = 0
  gives the mean of V; M = 1 gives V_0;
- loss invariants: 1 - cos in [0, 2]; zero when F is parallel to the target;
  the cosine gradient is orthogonal to F; the trust-region gradient is
  2 lambda (K - K0);
- central finite differences of the loss.
"""
import numpy as np
import pytest
import torch

from oracle import decode_oracle as DO


def _rand(seed, n=37, d=16, M=24, D=40):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, d))
    K = rng.standard_normal((M, d))
    V = rng.standard_normal((M, D))
    T = rng.standard_normal((n, D))
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    K0 = K + 0.01 * rng.standard_normal(K.shape)
    return Q, K, V, T, K0


@pytest.mark.parametrize("seed,d", [(0, 16), (1, 32), (2, 5)])
def test_forward_matches_library_attention(seed, d):
    Q, K, V, _, _ = _rand(seed, d=d)
    F, P, m, l = DO.decode_forward(Q, K, V)
    ref = torch.nn.functional.scaled_dot_product_attention(
        torch.from_numpy(Q)[None], torch.from_numpy(K)[None], torch.from_numpy(V)[None])[0]
    np.testing.assert_allclose(F, ref.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(P.sum(1), 1.0, rtol=1e-14)


def test_backward_matches_library_autograd():
    Q, K, V, _, _ = _rand(3, d=16)
    dF = np.random.default_rng(4).standard_normal((Q.shape[0], V.shape[1]))
    dQ, dK, dV = DO.decode_backward(Q, K, V, dF)
    tq, tk, tv = (torch.tensor(a, requires_grad=True) for a in (Q, K, V))
    out = torch.nn.functional.scaled_dot_product_attention(tq[None], tk[None], tv[None])[0]
    out.backward(torch.from_numpy(dF))
    np.testing.assert_allclose(dQ, tq.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dK, tk.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dV, tv.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_one_hot_row_returns_value_row_exactly():
    # Rows of K on a scaled orthonormal basis; Q_p = beta K_j puts a logit gap
    # far beyond exp underflow (745 in FP64), so P_p is exactly one-hot.
    rng = np.random.default_rng(5)
    d, M = 16, 12
    basis, _ = np.linalg.qr(rng.standard_normal((d, d)))
    K = 3.0 * basis[:M]
    V = rng.standard_normal((M, 33))
    js = np.array([0, 3, 7, 11, 5])
    Q = 400.0 * K[js]
    F, P, _, _ = DO.decode_forward(Q, K, V)
    assert np.array_equal(P, np.eye(M)[js])
    assert np.array_equal(F, V[js])


def test_zero_query_gives_mean_value():
    _, K, V, _, _ = _rand(6)
    F, P, _, _ = DO.decode_forward(np.zeros((4, K.shape[1])), K, V)
    np.testing.assert_allclose(F, np.tile(V.mean(0), (4, 1)), rtol=1e-13, atol=1e-14)


def test_single_atom_returns_it():
    Q, K, V, _, _ = _rand(7, M=1)
    F, _, _, _ = DO.decode_forward(Q, K, V)
    assert np.array_equal(F, np.tile(V[0], (Q.shape[0], 1)))


def test_cosine_loss_range_and_parallel_target():
    Q, K, V, T, K0 = _rand(8)
    c = DO.cosine(DO.decode_forward(Q, K, V)[0], T)
    assert np.all(1 - c >= 0) and np.all(1 - c <= 2)
    F = DO.decode_forward(Q, K, V)[0]
    Tpar = 2.5 * F
    r = DO.loss_and_grads(Q, K, V, Tpar, K, 0.1)
    assert abs(r["loss"]) < 1e-14
    r2 = DO.loss_and_grads(Q, K, V, -F, K, 0.0)
    assert r2["loss"] == pytest.approx(2.0, abs=1e-14)


def test_cosine_gradient_orthogonal_to_F():
    Q, K, V, T, K0 = _rand(9)
    r = DO.loss_and_grads(Q, K, V, T, K0, 0.1)
    dots = (r["gF"] * r["F"]).sum(1)
    scale = np.linalg.norm(r["gF"], axis=1) * np.linalg.norm(r["F"], axis=1)
    assert np.all(np.abs(dots) <= 1e-13 * scale)


def test_trust_region_gradient_closed_form():
    Q, K, V, T, K0 = _rand(10)
    r0 = DO.loss_and_grads(Q, K, V, T, K0, 0.0)
    r1 = DO.loss_and_grads(Q, K, V, T, K0, 0.1)
    np.testing.assert_allclose(r1["dK"] - r0["dK"], 0.2 * (K - K0), rtol=1e-12, atol=1e-15)
    assert r1["loss"] - r0["loss"] == pytest.approx(0.1 * ((K - K0) ** 2).sum(), rel=1e-12)


@pytest.mark.parametrize("which", ["Q", "K", "V"])
def test_loss_gradients_finite_differences(which):
    Q, K, V, T, K0 = _rand(11, n=9, d=8, M=6, D=10)
    lam = 0.1
    r = DO.loss_and_grads(Q, K, V, T, K0, lam)
    args = dict(Q=Q, K=K, V=V)
    grad = dict(Q=r["dQ"], K=r["dK"], V=r["dV"])[which]
    A = args[which]
    h = 1e-6
    fd = np.zeros_like(A)
    for idx in np.ndindex(A.shape):
        Ap, Am = A.copy(), A.copy()
        Ap[idx] += h
        Am[idx] -= h
        lp = DO.feature_loss(**{**args, which: Ap}, T=T, K0=K0, lambda_tr=lam)
        lm = DO.feature_loss(**{**args, which: Am}, T=T, K0=K0, lambda_tr=lam)
        fd[idx] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(grad, fd, rtol=1e-6, atol=1e-9)
