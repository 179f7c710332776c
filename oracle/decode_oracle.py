"""FP64 oracle for the dictionary decode and the feature loss.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.

What it computes:
  - Eq. 5 (Sec. III-B): reconstructed embeddings F = softmax(logits) V, in the
    untied form with a free key matrix K and value matrix V, logits
    S = Q K^T / sqrt(d) (d = query dimension).  Softmax is over the M
    dictionary atoms of each pixel row.
  - Eq. 6: the cosine term of the feature loss, 1 - cos(F_p, T_p) per pixel,
    averaged over the n pixels passed, plus a trust-region penalty on the
    dictionary keys, lambda_tr * ||K - K0||_F^2 (the configurations' squared
    Frobenius form of the paper's trust region; K0 is the initial K).
  - The exact gradients of that loss with respect to Q, K and V, by the chain
    rule through cosine, the weighted sum, the softmax and the logits.

The cosine denominator is guarded as max(||F_p|| ||T_p||, 1e-8).
Matrix products are library calls (numpy, FP64); nothing is blocked or fused.
"""
from __future__ import annotations

import numpy as np

COS_EPS = 1e-8


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def decode_forward(Q, K, V):
    """F = softmax(Q K^T / sqrt(d)) V.  Returns (F, P, m, l): P the attention
    weights, m the row max of the logits, l the row sum of exp(S - m)."""
    Q, K, V = _f64(Q), _f64(K), _f64(V)
    d = Q.shape[1]
    S = (Q @ K.T) / np.sqrt(d)
    m = S.max(axis=1)
    E = np.exp(S - m[:, None])
    l = E.sum(axis=1)
    P = E / l[:, None]
    F = P @ V
    return F, P, m, l


def cosine(F, T):
    """Per-row cosine similarity with the guarded denominator."""
    F, T = _f64(F), _f64(T)
    den = np.maximum(np.linalg.norm(F, axis=1) * np.linalg.norm(T, axis=1), COS_EPS)
    return (F * T).sum(axis=1) / den


def feature_loss(Q, K, V, T, K0, lambda_tr):
    """L = mean_p (1 - cos(F_p, T_p)) + lambda_tr ||K - K0||^2."""
    F, _, _, _ = decode_forward(Q, K, V)
    c = cosine(F, T)
    tr = float(lambda_tr) * float(((_f64(K) - _f64(K0)) ** 2).sum())
    return float((1.0 - c).mean()) + tr


def decode_backward(Q, K, V, dF):
    """Gradients of <dF, F> with respect to Q, K, V (the adjoint of Eq. 5)."""
    Q, K, V, dF = _f64(Q), _f64(K), _f64(V), _f64(dF)
    d = Q.shape[1]
    _, P, _, _ = decode_forward(Q, K, V)
    dV = P.T @ dF
    dP = dF @ V.T
    delta = (P * dP).sum(axis=1)
    dS = P * (dP - delta[:, None])
    dQ = (dS @ K) / np.sqrt(d)
    dK = (dS.T @ Q) / np.sqrt(d)
    return dQ, dK, dV


def loss_and_grads(Q, K, V, T, K0, lambda_tr):
    """Loss of Eq. 6 (cosine + trust region) and its exact gradients.

    Returns dict(loss, F, cos, dQ, dK, dV, gF) where gF = dL/dF."""
    Q, K, V, T, K0 = _f64(Q), _f64(K), _f64(V), _f64(T), _f64(K0)
    n = Q.shape[0]
    F, P, m, l = decode_forward(Q, K, V)
    nF = np.linalg.norm(F, axis=1)
    nT = np.linalg.norm(T, axis=1)
    raw = nF * nT
    den = np.maximum(raw, COS_EPS)
    c = (F * T).sum(axis=1) / den
    loss = float((1.0 - c).mean()) + float(lambda_tr) * float(((K - K0) ** 2).sum())
    # d c / d F: T/den - c F/|F|^2 where the guard is inactive; T/den where it is.
    active = raw > COS_EPS
    safe_nF2 = np.where(nF > 0, nF * nF, 1.0)
    dcdF = T / den[:, None] - np.where(active, c / safe_nF2, 0.0)[:, None] * F
    gF = -dcdF / n
    dQ, dK, dV = decode_backward(Q, K, V, gF)
    dK = dK + 2.0 * float(lambda_tr) * (K - K0)
    return dict(loss=loss, F=F, P=P, m=m, l=l, cos=c, dQ=dQ, dK=dK, dV=dV, gF=gF)
