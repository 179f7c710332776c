"""A CPU model of the FP8 forward arithmetic (test code, not the oracle).

Rounds exactly where the FP8 kernel rounds: BF16 Q and K for the logits, OCP
E4M3 (3 mantissa bits, bias 7, max 448, subnormals to 2^-9, round to nearest
even) for V / s^V, and the max-normalised weights times the folded V scales
as two E4M3 terms (the rounded value plus the rounded residual); everything
else in FP64.  Used to check that the kernel implements the
documented quantisation, separately from how far that quantisation is from
the exact result.
"""
import numpy as np


def e4m3(x):
    x = np.asarray(x, np.float64)
    s = np.sign(x)
    a = np.minimum(np.abs(x), 448.0)
    e = np.maximum(np.floor(np.log2(np.maximum(a, 2.0 ** -12))), -6)
    step = 2.0 ** (e - 3)
    return s * np.minimum(np.round(a / step) * step, 448.0)


def bf16(x):
    x = np.ascontiguousarray(np.asarray(x, np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def fp8_forward(Q, K, V):
    d = Q.shape[1]
    S = bf16(Q) @ bf16(K).T / np.sqrt(d)
    Pt = np.exp(S - S.max(1, keepdims=True))
    l = Pt.sum(1, keepdims=True)
    sV = np.abs(np.asarray(V, np.float64)).max(1) / 448.0
    vmax = sV.max()
    V8 = e4m3(np.asarray(V, np.float64) / np.where(sV > 0, sV, 1.0)[:, None])
    q = Pt * (sV * 448.0 / vmax)[None, :]
    hi = e4m3(q)
    P8 = hi + e4m3(q - hi)
    return (P8 @ V8) * (vmax / 448.0) / l
