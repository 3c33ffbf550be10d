"""Binary64 image-quality metrics for reporting reconstructions.

PSNR with a stated data range, and SSIM following Wang, Bovik, Sheikh &
Simoncelli, "Image quality assessment: from error visibility to structural
similarity", IEEE TIP 13(4), 2004: local means, variances and covariance under
an 11 x 11 Gaussian window (sigma 1.5), constants C1 = (0.01 L)^2,
C2 = (0.03 L)^2, SSIM map averaged over the valid region.  3-D inputs
(videos, time last) average SSIM over frames.
"""
import numpy as np
from scipy import ndimage


def psnr(x, ref, data_range=1.0):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    mse = np.mean((x - ref) ** 2)
    if mse == 0:
        return float("inf")
    return float(10.0 * np.log10(data_range ** 2 / mse))


def _gaussian_window(size=11, sigma=1.5):
    ax = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-ax ** 2 / (2 * sigma ** 2))
    w = np.outer(g, g)
    return w / w.sum()


def _ssim2d(x, y, data_range, win):
    c1 = (0.01 * data_range) ** 2
    c2 = (0.03 * data_range) ** 2
    f = lambda a: ndimage.correlate(a, win, mode="reflect")
    mx, my = f(x), f(y)
    sxx = f(x * x) - mx * mx
    syy = f(y * y) - my * my
    sxy = f(x * y) - mx * my
    m = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    h = win.shape[0] // 2
    return float(m[h:-h, h:-h].mean()) if min(x.shape) > 2 * h else float(m.mean())


def ssim(x, ref, data_range=1.0):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    win = _gaussian_window()
    if x.ndim == 2:
        return _ssim2d(x, ref, data_range, win)
    if x.ndim == 3:
        return float(np.mean([_ssim2d(x[..., t], ref[..., t], data_range, win)
                              for t in range(x.shape[-1])]))
    raise ValueError("ssim takes 2-D images or 3-D (time last) videos")
