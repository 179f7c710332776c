"""FP64 oracle for the paper's tied dictionary decode and full feature loss.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark, never by
the product path.  It shares no code with the GPU library.

What it computes (Sec. III-C, Eq. 5 and Eq. 6 as the paper states them):
  - The decode F^ = Softmax(Q W D^T) D with the softmax taken over the cosine
    similarity of the rows of Q W and the dictionary atoms D_j, each normalised
    to unit length, divided by a temperature tau:
        C[p][j] = <x_p / |x_p|, D_j / |D_j|>,  x_p = Q_p W,
        P = softmax_j(C / tau),                F^ = P D.
    Norms are guarded as max(|.|, 1e-12) (a zero row normalises to zero).
  - The feature loss
        L = lambda_cos * mean_p (1 - cos(F^_p, F_p))
          + lambda_2   * mean_p |F^_p - F_p|^2
          + lambda_D   * sum_j ReLU(|D0_j - D_j| - delta),
    with the cosine denominator guarded as max(|F^_p| |F_p|, 1e-8).
  - Its exact gradients with respect to Q, W and D, by the chain rule written
    out step by step (cosine / L2 -> weighted sum -> softmax -> cosine logits
    -> row normalisations -> the products Q W and the normalised D).

Matrix products are numpy calls in FP64; nothing is blocked or fused.
"""
from __future__ import annotations

import numpy as np

NORM_EPS = 1e-12
COS_EPS = 1e-8


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def _normalize_rows(X):
    """X / max(|X_row|, eps) and the guarded norms."""
    n = np.linalg.norm(X, axis=1)
    g = np.maximum(n, NORM_EPS)
    return X / g[:, None], n, g


def _normalize_rows_backward(dA, A, n, g):
    """Adjoint of A = X / max(|X|, eps): (dA - A <A, dA>) / |X| where the guard
    is inactive, dA / eps where it is."""
    active = n > NORM_EPS
    proj = np.where(active, (A * dA).sum(axis=1), 0.0)
    return (dA - A * proj[:, None]) / g[:, None]


def tied_forward(Q, W, D, tau):
    """F^ = softmax(cos(QW, D) / tau) D.  Returns (F, P, C)."""
    Q, W, D = _f64(Q), _f64(W), _f64(D)
    A, _, _ = _normalize_rows(Q @ W)
    B, _, _ = _normalize_rows(D)
    C = A @ B.T
    S = C / float(tau)
    E = np.exp(S - S.max(axis=1, keepdims=True))
    P = E / E.sum(axis=1, keepdims=True)
    return P @ D, P, C


def tied_loss(Q, W, D, T, D0, tau, lam_cos, lam_2, lam_D, delta):
    F, _, _ = tied_forward(Q, W, D, tau)
    F, T = _f64(F), _f64(T)
    den = np.maximum(np.linalg.norm(F, axis=1) * np.linalg.norm(T, axis=1), COS_EPS)
    c = (F * T).sum(axis=1) / den
    dev = np.linalg.norm(_f64(D0) - _f64(D), axis=1)
    return float(lam_cos * (1.0 - c).mean() + lam_2 * ((F - T) ** 2).sum(axis=1).mean()
                 + lam_D * np.maximum(dev - delta, 0.0).sum())


def tied_loss_and_grads(Q, W, D, T, D0, tau, lam_cos, lam_2, lam_D, delta):
    """Loss of Eq. 6 with the decode of Eq. 5, and dL/dQ, dL/dW, dL/dD.

    Returns dict(loss, F, P, cos, dQ, dW, dD, gF, parts) where gF = dL/dF^ and
    parts = (cosine term, L2 term, trust-region term)."""
    Q, W, D, T, D0 = _f64(Q), _f64(W), _f64(D), _f64(T), _f64(D0)
    n = Q.shape[0]
    tau = float(tau)
    # forward, keeping the intermediates
    X = Q @ W
    A, nx, gx = _normalize_rows(X)
    B, nd, gd = _normalize_rows(D)
    S = (A @ B.T) / tau
    E = np.exp(S - S.max(axis=1, keepdims=True))
    P = E / E.sum(axis=1, keepdims=True)
    F = P @ D
    nF = np.linalg.norm(F, axis=1)
    nT = np.linalg.norm(T, axis=1)
    raw = nF * nT
    den = np.maximum(raw, COS_EPS)
    c = (F * T).sum(axis=1) / den
    dev = np.linalg.norm(D0 - D, axis=1)
    parts = (float(lam_cos * (1.0 - c).mean()), float(lam_2 * ((F - T) ** 2).sum(axis=1).mean()),
             float(lam_D * np.maximum(dev - delta, 0.0).sum()))
    loss = sum(parts)
    # dL/dF^: the cosine term (guard as in the untied oracle) and the L2 term
    active = raw > COS_EPS
    safe_nF2 = np.where(nF > 0, nF * nF, 1.0)
    dcdF = T / den[:, None] - np.where(active, c / safe_nF2, 0.0)[:, None] * F
    gF = -lam_cos * dcdF / n + 2.0 * lam_2 * (F - T) / n
    # F^ = P D
    dD = P.T @ gF
    dP = gF @ D.T
    # softmax
    dS = P * (dP - (P * dP).sum(axis=1, keepdims=True))
    # S = A B^T / tau
    dA = (dS @ B) / tau
    dB = (dS.T @ A) / tau
    # the row normalisations
    dX = _normalize_rows_backward(dA, A, nx, gx)
    dD += _normalize_rows_backward(dB, B, nd, gd)
    # X = Q W
    dQ = dX @ W.T
    dW = Q.T @ dX
    # trust region: lambda_D (D - D0) / |D - D0| outside the radius delta
    outside = dev > delta
    safe_dev = np.where(outside, dev, 1.0)
    dD += lam_D * np.where(outside, 1.0 / safe_dev, 0.0)[:, None] * (D - D0)
    return dict(loss=loss, F=F, P=P, cos=c, dQ=dQ, dW=dW, dD=dD, gF=gF, parts=parts)
