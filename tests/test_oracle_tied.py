"""Pins of the FP64 oracle for the tied decode and the full feature loss
(Eq. 5-6): an independent torch-autograd formulation, finite differences,
closed forms and special cases."""
import numpy as np
import pytest

from oracle import tied_decode_oracle as TD

torch = pytest.importorskip("torch")

PARAMS = dict(tau=0.1, lam_cos=0.5, lam_2=0.5, lam_D=0.2, delta=0.1)


def _inputs(seed, n=37, ds=16, M=24, df=40, dev_scale=0.08):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, ds))
    W = rng.standard_normal((ds, df)) / np.sqrt(ds)
    D0 = rng.standard_normal((M, df))
    D = D0 + dev_scale * rng.standard_normal((M, df))
    T = rng.standard_normal((n, df))
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    return Q, W, D, T, D0


def _torch_loss(Q, W, D, T, D0, tau, lam_cos, lam_2, lam_D, delta):
    """The same loss written with torch ops, differentiated by autograd."""
    x = torch.nn.functional.normalize(Q @ W, dim=1, eps=1e-12)
    b = torch.nn.functional.normalize(D, dim=1, eps=1e-12)
    P = torch.softmax((x @ b.T) / tau, dim=1)
    F = P @ D
    cos = (F * T).sum(1) / torch.clamp(F.norm(dim=1) * T.norm(dim=1), min=1e-8)
    l2 = ((F - T) ** 2).sum(1).mean()
    tr = torch.relu((D0 - D).norm(dim=1) - delta).sum()
    return lam_cos * (1 - cos).mean() + lam_2 * l2 + lam_D * tr


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_torch_autograd_fp64(seed):
    Q, W, D, T, D0 = _inputs(seed)
    r = TD.tied_loss_and_grads(Q, W, D, T, D0, **PARAMS)
    tq, tw, td = (torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (Q, W, D))
    L = _torch_loss(tq, tw, td, torch.tensor(T), torch.tensor(D0), **PARAMS)
    L.backward()
    assert abs(L.item() - r["loss"]) < 1e-12 * max(1.0, abs(r["loss"]))
    for name, t in (("dQ", tq), ("dW", tw), ("dD", td)):
        np.testing.assert_allclose(r[name], t.grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=name)


def test_finite_differences():
    Q, W, D, T, D0 = _inputs(3, n=9, ds=16, M=7, df=12, dev_scale=0.2)
    r = TD.tied_loss_and_grads(Q, W, D, T, D0, **PARAMS)
    rng = np.random.default_rng(4)
    h = 1e-6
    for name, arr in (("dQ", Q), ("dW", W), ("dD", D)):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            a1, a2 = arr.copy(), arr.copy()
            a1[idx] += h
            a2[idx] -= h
            args = {"dQ": (a1, W, D), "dW": (Q, a1, D), "dD": (Q, W, a1)}[name]
            args2 = {"dQ": (a2, W, D), "dW": (Q, a2, D), "dD": (Q, W, a2)}[name]
            fd = (TD.tied_loss(*args, T, D0, **PARAMS) - TD.tied_loss(*args2, T, D0, **PARAMS)) / (2 * h)
            assert abs(fd - r[name][idx]) < 1e-6 * max(1.0, abs(fd)), (name, idx, fd, r[name][idx])


def test_single_atom_returns_it():
    Q, W, D, T, D0 = _inputs(5, M=1)
    F, P, _ = TD.tied_forward(Q, W, D, 0.1)
    assert np.all(P == 1.0)
    np.testing.assert_array_equal(F, np.repeat(D, Q.shape[0], axis=0))


def test_sharp_temperature_selects_the_aligned_atom():
    # D has orthonormal rows (scaled); Q W points along atom 3: with a small
    # temperature the attention is one-hot and F^ is that atom exactly.
    df, M, ds = 8, 5, 8
    D = 2.0 * np.eye(M, df)
    W = np.eye(ds, df)
    Q = np.zeros((1, ds))
    Q[0, 3] = 0.7
    F, P, C = TD.tied_forward(Q, W, D, 1e-3)
    np.testing.assert_allclose(C[0], np.eye(M)[3])
    np.testing.assert_allclose(P[0], np.eye(M)[3], atol=1e-300)
    np.testing.assert_allclose(F[0], D[3])


def test_zero_query_gives_the_mean_atom():
    Q, W, D, _, _ = _inputs(6)
    Q[2] = 0.0
    F, P, _ = TD.tied_forward(Q, W, D, 0.1)
    np.testing.assert_allclose(P[2], np.full(D.shape[0], 1.0 / D.shape[0]))
    np.testing.assert_allclose(F[2], D.mean(axis=0))


def test_trust_region_hinge():
    Q, W, D0, T, _ = _inputs(7, dev_scale=0.0)
    D = D0.copy()
    v = np.zeros(D.shape[1])
    v[0] = 0.05                      # inside the radius: no penalty, no gradient
    D[0] += v
    w = np.zeros(D.shape[1])
    w[1], w[2] = 0.3, 0.4            # |w| = 0.5 > delta
    D[1] += w
    p = dict(PARAMS, lam_cos=0.0, lam_2=0.0)
    r = TD.tied_loss_and_grads(Q, W, D, T, D0, **p)
    assert abs(r["parts"][2] - 0.2 * (0.5 - 0.1)) < 1e-15
    np.testing.assert_allclose(r["dD"][0], 0.0, atol=1e-15)
    np.testing.assert_allclose(r["dD"][1], 0.2 * w / 0.5)
    np.testing.assert_allclose(r["dD"][2:], 0.0, atol=1e-15)


def test_reassociated_form_used_by_the_kernels():
    """The cosine logits equal Q' K^T with Q'_p = Q_p / (tau |Q_p W|) and
    K = normalize_rows(D) W^T, so the untied decode with V = D and logit scale 1
    computes the tied form (the mapping the GPU path relies on)."""
    Q, W, D, _, _ = _inputs(8)
    tau = 0.1
    Fo, _, C = TD.tied_forward(Q, W, D, tau)
    Qp = Q / (tau * np.linalg.norm(Q @ W, axis=1, keepdims=True))
    K = (D / np.linalg.norm(D, axis=1, keepdims=True)) @ W.T
    S = Qp @ K.T
    np.testing.assert_allclose(S, C / tau, rtol=1e-12, atol=1e-12)
    E = np.exp(S - S.max(1, keepdims=True))
    np.testing.assert_allclose((E / E.sum(1, keepdims=True)) @ D, Fo, rtol=1e-12)
