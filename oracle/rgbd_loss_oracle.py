"""FP64 oracle for the L1 colour and depth terms of the mapping objective.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark, never by
the product path.  It shares no code with the GPU library.

Eq. 7 takes the L1 norm of the rendered minus the observed image, Eq. 8 the L1
norm of the rendered minus the observed depth, and Eq. 9 weighs them.  Read as
means: the colour term over the 3 n colour values, the depth term over the
pixels that have an observed depth (> 0; a depth sensor leaves holes).  The
derivative of |x| is taken as sign(x), zero at x = 0.  The SSIM part of Eq. 7
is not computed.
"""
from __future__ import annotations

import numpy as np


def l1_losses(rgb, rgb_obs, depth, depth_obs, lambda_rgb, lambda_depth):
    """Returns dict(loss, d_rgb, d_depth, rgb_term, depth_term, n_valid)."""
    rgb, rgb_obs = np.asarray(rgb, np.float64), np.asarray(rgb_obs, np.float64)
    depth, depth_obs = np.asarray(depth, np.float64), np.asarray(depth_obs, np.float64)
    n = depth.shape[0]
    dI = rgb - rgb_obs
    dZ = depth - depth_obs
    valid = depth_obs > 0
    cnt = int(valid.sum())
    rgb_term = lambda_rgb * np.abs(dI).sum() / (3 * n) if n > 0 else 0.0
    depth_term = lambda_depth * np.abs(dZ[valid]).sum() / cnt if cnt > 0 else 0.0
    d_rgb = lambda_rgb * np.sign(dI) / (3 * max(n, 1))
    d_depth = np.where(valid, lambda_depth * np.sign(dZ) / max(cnt, 1), 0.0)
    return dict(loss=float(rgb_term + depth_term), d_rgb=d_rgb, d_depth=d_depth, rgb_term=float(rgb_term),
                depth_term=float(depth_term), n_valid=cnt)
