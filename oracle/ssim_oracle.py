"""FP64 oracle for the SSIM term of the photometric loss (Eq. 7).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark, never by
the product path.  It shares no code with the GPU library.

Eq. 7 adds lambda_I2 L_SSIM(I^, I) to the L1 colour term; the paper gives no
window or constants and builds on 3D Gaussian Splatting, whose SSIM loss is
read here: the structural similarity of Wang et al. per colour channel with an
11 x 11 Gaussian window of standard deviation 1.5 (normalised to sum 1),
C1 = 0.01^2, C2 = 0.03^2 and zero padding at the image border,

    mu_x = W * x,  sigma_x^2 = W * x^2 - mu_x^2,  sigma_xy = W * (x y) - mu_x mu_y,
    S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),

and L_SSIM = 1 - mean of S over every pixel and channel of every view (each
view is its own image; windows never cross views).  The gradient with respect
to the rendered image x is the chain rule written out: the per-pixel partial
derivatives of S with respect to mu_x, W * x^2 and W * (x y), each spread back
by the same window (the window is symmetric, so the adjoint of the zero-padded
filter is the filter itself).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5


def window():
    k = np.arange(WINDOW) - WINDOW // 2
    g = np.exp(-(k * k) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def _filt(img):
    """Zero-padded windowed sum of one [H, W] image."""
    return ndimage.correlate(img, window(), mode="constant", cval=0.0)


def ssim_view(x, y):
    """x, y [H, W, 3] -> (S [H, W, 3], intermediates)."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    S = np.empty_like(x)
    parts = []
    for c in range(x.shape[2]):
        xc, yc = x[..., c], y[..., c]
        mx, my = _filt(xc), _filt(yc)
        exx, eyy, exy = _filt(xc * xc), _filt(yc * yc), _filt(xc * yc)
        sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
        a1, a2 = 2 * mx * my + C1, 2 * sxy + C2
        b1, b2 = mx * mx + my * my + C1, sxx + syy + C2
        S[..., c] = a1 * a2 / (b1 * b2)
        parts.append((mx, my, a1, a2, b1, b2))
    return S, parts


def ssim_loss(rgb, rgb_obs, sizes):
    """rgb, rgb_obs [P, 3]: views concatenated, each row-major [H, W]; sizes a
    list of (W, H).  Returns dict(loss, d_rgb, mean_ssim)."""
    rgb, rgb_obs = np.asarray(rgb, np.float64), np.asarray(rgb_obs, np.float64)
    total = 3 * sum(w * h for w, h in sizes)
    grad = np.zeros_like(rgb)
    ssum = 0.0
    off = 0
    for w, h in sizes:
        x = rgb[off:off + w * h].reshape(h, w, 3)
        y = rgb_obs[off:off + w * h].reshape(h, w, 3)
        S, parts = ssim_view(x, y)
        ssum += S.sum()
        g = np.empty_like(x)
        for c, (mx, my, a1, a2, b1, b2) in enumerate(parts):
            s = S[..., c]
            dS = -1.0 / total  # dL/dS at every pixel
            # S = a1 a2 / (b1 b2) with a1(mu_x), a2(E_xy, mu_x), b1(mu_x), b2(E_xx, mu_x)
            d_mx = dS * ((2 * my * a2 - 2 * my * a1) / (b1 * b2) - s * (2 * mx / b1 - 2 * mx / b2))
            d_exx = dS * (-s / b2)
            d_exy = dS * (2 * a1 / (b1 * b2))
            xc, yc = x[..., c], y[..., c]
            g[..., c] = _filt(d_mx) + 2 * xc * _filt(d_exx) + yc * _filt(d_exy)
        grad[off:off + w * h] = g.reshape(-1, 3)
        off += w * h
    mean = ssum / total if total else 0.0
    return dict(loss=1.0 - mean, d_rgb=grad, mean_ssim=mean)
