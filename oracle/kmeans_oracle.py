"""FP64 oracle for the streaming K-means dictionary initialisation (Eq. 10).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark, never by
the product path.  It shares no code with the GPU library.

What it computes (Sec. III-D, Eq. 10, read as the streaming K-means of
O'Callaghan et al. that the paper cites):

  D_t0 = StreamKMeans(F_t, D_{t-1}, K)

  1. Local K-means ("micro-factors"): the keyframe's embeddings F_t [n, D]
     (each of weight 1) are summarised into m micro-centres by Lloyd's
     iteration started from m of the embeddings, F_t[s] (the indices s are the
     random draw, passed in).  Each micro-centre carries as weight the number
     of embeddings assigned to it in the last iteration.
  2. Merge: the weighted micro-centres join the current global centres
     D_{t-1} [Kp, D] with their weights w_{t-1}.
  3. Re-cluster: weighted Lloyd's iteration of the merged set into K centres,
     started from D_{t-1} followed by the first K - Kp micro-centres.  The
     output weights are the total weight assigned to each centre in the last
     iteration.

One Lloyd iteration: every point goes to its nearest centre in squared
Euclidean distance (ties to the lowest centre index); every centre moves to
the weighted mean of its points; a centre with no points (or zero total
weight) stays where it is.  The iteration counts are fixed (no convergence
test).

Distances are the plain definition sum_d (x_d - c_d)^2, evaluated in FP64 in
chunks of points; nothing is reassociated into dot products.
"""
from __future__ import annotations

import numpy as np

_CHUNK_ELEMS = 1 << 24


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def sqdist(X, C):
    """[n, k] squared Euclidean distances, straight from the definition."""
    X, C = _f64(X), _f64(C)
    n, k = X.shape[0], C.shape[0]
    out = np.empty((n, k))
    rows = max(1, _CHUNK_ELEMS // max(1, k * X.shape[1]))
    for i in range(0, n, rows):
        diff = X[i:i + rows, None, :] - C[None, :, :]
        out[i:i + rows] = (diff * diff).sum(axis=2)
    return out


def assign(X, C):
    """Nearest centre of every point (lowest index on ties).

    Returns (a, d2, margin): the centre index, the squared distance to it, and
    the gap to the second nearest centre (inf with one centre)."""
    d = sqdist(X, C)
    if d.shape[0] == 0:
        return np.zeros(0, np.int64), np.zeros(0), np.zeros(0)
    a = np.argmin(d, axis=1)
    best = d[np.arange(d.shape[0]), a]
    if d.shape[1] > 1:
        part = np.partition(d, 1, axis=1)
        margin = part[:, 1] - part[:, 0]
    else:
        margin = np.full(d.shape[0], np.inf)
    return a, best, margin


def update(X, w, a, C):
    """Weighted means of the assigned points; empty centres keep C.

    Returns (C_new, W) with W the total weight per centre."""
    X, C = _f64(X), _f64(C)
    k = C.shape[0]
    w = np.ones(X.shape[0]) if w is None else _f64(w)
    S = np.zeros_like(C)
    W = np.zeros(k)
    np.add.at(S, a, w[:, None] * X)
    np.add.at(W, a, w)
    C_new = C.copy()
    nz = W > 0
    C_new[nz] = S[nz] / W[nz, None]
    return C_new, W


def lloyd(X, w, C0, iters):
    """``iters`` Lloyd iterations from C0.  Returns (C, W, a) where a is the
    last assignment and W the total weight per centre under it."""
    if iters < 1:
        raise ValueError("iters must be >= 1")
    C = _f64(C0).copy()
    for _ in range(iters):
        a, _, _ = assign(X, C)
        C, W = update(X, w, a, C)
    return C, W, a


def cost(X, w, C):
    """Weighted K-means objective sum_i w_i min_j |x_i - c_j|^2."""
    _, d2, _ = assign(X, C)
    w = np.ones(len(d2)) if w is None else _f64(w)
    return float((w * d2).sum())


def stream_kmeans(F, D_prev, w_prev, K, seeds, iters_local, iters_global):
    """Eq. 10 as read above.  Returns dict(D, W, micro, micro_w, a_micro).

    F [n, D] new embeddings; D_prev [Kp, D] and w_prev [Kp] the global centres
    and their weights (Kp = 0 on the first keyframe); seeds [m] distinct
    indices into F; requires Kp <= K and m >= K - Kp."""
    F = _f64(F)
    D_prev = _f64(D_prev).reshape(-1, F.shape[1])
    w_prev = _f64(w_prev).reshape(-1)
    seeds = np.asarray(seeds, dtype=np.int64)
    Kp, m = D_prev.shape[0], seeds.shape[0]
    if Kp > K or m < K - Kp:
        raise ValueError("need Kp <= K and m >= K - Kp")
    if m > 0:
        micro, micro_w, a_micro = lloyd(F, None, F[seeds], iters_local)
    else:
        micro, micro_w, a_micro = np.zeros((0, F.shape[1])), np.zeros(0), np.zeros(0, np.int64)
    P = np.concatenate([D_prev, micro], axis=0)
    Pw = np.concatenate([w_prev, micro_w])
    G0 = np.concatenate([D_prev, micro[:K - Kp]], axis=0)
    G, W, _ = lloyd(P, Pw, G0, iters_global)
    return dict(D=G, W=W, micro=micro, micro_w=micro_w, a_micro=a_micro)
