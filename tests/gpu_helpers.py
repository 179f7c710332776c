"""Shared helpers of the GPU parity tests."""
from __future__ import annotations

import sys

import numpy as np

# A pixel is "ambiguous" when the oracle's FP64 walk takes a threshold decision
# (alpha skip, alpha clamp, termination) within this relative distance of the
# threshold; the FP32 kernel may then legitimately take the other branch.
AMBIGUOUS = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(x, ref) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))


def to_np(t):
    return t.detach().float().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def ws_u32(ws, ptr: int, count: int) -> np.ndarray:
    """``count`` uint32 at device address ``ptr`` inside the workspace tensor ``ws``."""
    import torch
    off = int(ptr) - ws.data_ptr()
    assert 0 <= off and off % 4 == 0 and off + 4 * count <= ws.numel(), (off, count, ws.numel())
    return ws[off:off + 4 * count].view(torch.int32).cpu().numpy().view(np.uint32)
