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


# An element may be off by at most this many times the L2 bar, relative to the
# largest reference element: a few badly wrong elements among many correct
# ones fail a bar that the L2 norm alone would let through.
ELEM_FACTOR = 10.0


class Err(float):
    """Relative L2 error ||x - ref|| / ||ref|| (the float value) together with
    the largest element error max |x - ref| / max |ref| (``.elem``).  ``e < bar``
    holds only when both are within their bars: the L2 error below ``bar`` and
    the element error below ``ELEM_FACTOR * bar``."""

    def __new__(cls, l2: float, elem: float):
        o = float.__new__(cls, l2)
        o.elem = elem
        return o

    def __lt__(self, bar):
        return float(self) < bar and self.elem < ELEM_FACTOR * bar

    def __le__(self, bar):
        return float(self) <= bar and self.elem <= ELEM_FACTOR * bar

    def __format__(self, spec):
        return f"{float(self):{spec}} (elem {self.elem:{spec}})" if spec else f"{float(self)} (elem {self.elem})"


def rel_err(x, ref) -> Err:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    d = np.abs(x - ref)
    big = float(np.abs(ref).max()) if ref.size else 0.0
    elem = float(d.max() / big) if d.size and big > 0 else (float(d.max()) if d.size else 0.0)
    l2 = float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))
    return Err(l2, elem)


def to_np(t):
    return t.detach().float().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def ws_u32(ws, ptr: int, count: int) -> np.ndarray:
    """``count`` uint32 at device address ``ptr`` inside the workspace tensor ``ws``."""
    import torch
    off = int(ptr) - ws.data_ptr()
    assert 0 <= off and off % 4 == 0 and off + 4 * count <= ws.numel(), (off, count, ws.numel())
    return ws[off:off + 4 * count].view(torch.int32).cpu().numpy().view(np.uint32)
