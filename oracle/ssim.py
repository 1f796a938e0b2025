"""FP64 oracle of the D-SSIM part of the colour loss (Sec. 3.3, Eq. of L_color; App. A).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU-baseline leg; it
shares no code with the GPU path.

The paper weights a D-SSIM term against the L1 term of the colour loss of every layer,
L^l = (1 - lambda_ssim) |C^l - C_gt|_1 + lambda_ssim L_D-SSIM(C^l, C_gt), and names the
metric with a citation but no formula. Reading used here (the structural-similarity index
with a Gaussian window, as in the 3D Gaussian Splatting training code the paper builds on):
  * per colour channel, an 11 x 11 Gaussian window with sigma 1.5, normalised to sum 1,
    applied as a 'same'-size convolution with zeros outside the image (so the window is
    separable: one 11-tap pass along rows, one along columns);
  * mu_x = G*x, mu_y = G*y, s_xx = G*(x x) - mu_x^2, s_yy = G*(y y) - mu_y^2,
    s_xy = G*(x y) - mu_x mu_y, with C1 = 0.01^2 and C2 = 0.03^2 (colours in [0, 1]);
  * SSIM(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2));
  * L_D-SSIM = 1 - mean over pixels and channels of SSIM.
The L1 term is the mean absolute difference over pixels and channels; the loss of a render
sums lambda^l L^l over frames, views and layers.

Gradient: with S written in terms of mu_x, E_xx = G*(x x) and E_xy = G*(x y), the derivative
of sum_p w(p) S(p) with respect to x(q) is (G*a)(q) + 2 x(q) (G*b)(q) + y(q) (G*c)(q) where
a = w dS/dmu_x, b = w dS/dE_xx, c = w dS/dE_xy; G* with zero padding is its own adjoint
because the window is symmetric.
"""
from __future__ import annotations

import numpy as np

WIN = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d() -> np.ndarray:
    x = np.arange(WIN, dtype=np.float64) - WIN // 2
    g = np.exp(-x * x / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def blur(img: np.ndarray) -> np.ndarray:
    """Separable Gaussian window over the last two axes, zero outside the image, FP64."""
    img = np.asarray(img, np.float64)
    g = window_1d()
    r = WIN // 2
    H, W = img.shape[-2:]
    pad = np.zeros(img.shape[:-2] + (H, W + 2 * r))
    pad[..., r:r + W] = img
    h = sum(g[k] * pad[..., k:k + W] for k in range(WIN))
    pad = np.zeros(img.shape[:-2] + (H + 2 * r, W))
    pad[..., r:r + H, :] = h
    return sum(g[k] * pad[..., k:k + H, :] for k in range(WIN))


def ssim_parts(x: np.ndarray, y: np.ndarray):
    """SSIM map of x against y and its partial derivatives with respect to mu_x, E_xx, E_xy."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mu1, mu2 = blur(x), blur(y)
    exx, eyy, exy = blur(x * x), blur(y * y), blur(x * y)
    s11, s22, s12 = exx - mu1 * mu1, eyy - mu2 * mu2, exy - mu1 * mu2
    a1 = 2.0 * mu1 * mu2 + C1
    a2 = 2.0 * s12 + C2
    b1 = mu1 * mu1 + mu2 * mu2 + C1
    b2 = s11 + s22 + C2
    S = a1 * a2 / (b1 * b2)
    d_mu1 = (2.0 * mu2 * a2 - 2.0 * mu2 * a1) / (b1 * b2) - S * (2.0 * mu1 / b1 - 2.0 * mu1 / b2)
    d_exx = -S / b2
    d_exy = 2.0 * a1 / (b1 * b2)
    return S, d_mu1, d_exx, d_exy


def ssim(x, y) -> float:
    return float(ssim_parts(x, y)[0].mean())


def color_loss(image: np.ndarray, target: np.ndarray, level_weights, lambda_ssim: float):
    """Layer-weighted colour loss and dL/dC. image [B][L][3][H][W], target [B][3][H][W]."""
    image = np.asarray(image, np.float64)
    target = np.asarray(target, np.float64)
    B, L, C, H, W = image.shape
    n = C * H * W
    loss = 0.0
    grad = np.zeros_like(image)
    for b in range(B):
        y = target[b]
        for l in range(L):
            x = image[b, l]
            w = float(level_weights[l])
            S, a, bb, cc = ssim_parts(x, y)
            loss += w * ((1.0 - lambda_ssim) * np.abs(x - y).mean() + lambda_ssim * (1.0 - S.mean()))
            g = w * (1.0 - lambda_ssim) * np.sign(x - y) / n
            coef = -w * lambda_ssim / n
            g += coef * (blur(a) + 2.0 * x * blur(bb) + y * blur(cc))
            grad[b, l] = g
    return loss, grad
