"""Reference of the point-cloud-to-voxel conversion and of the image-quality
figures (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; it shares no code with the HIP library.

Algorithm 1 of SlingBAG Pro ends by converting the point cloud to a voxel
grid; section 2 and Table 1 judge reconstructions by MSE, PSNR and SSIM
against the ground truth.  Written here in FP64 from their definitions:
the voxel value is the sum of the balls' initial-pressure profiles (section
4.1) at the voxel centre; SSIM is Wang et al.'s index with an 11-tap Gaussian
window (sigma 1.5) applied separably in 3-D over the voxels whose window lies
inside the volume.
"""
from __future__ import annotations

import numpy as np

GAUSS, UNIFORM = 1, 0


def voxelize(balls, grid, profile=GAUSS, K=5.0):
    """Volume [nx][ny][nz]: sum over balls of p0 * fhat(|c - r| / a) at voxel centres c."""
    vol = np.zeros((grid.nx, grid.ny, grid.nz))
    cx = grid.ox + (np.arange(grid.nx) + 0.5) * grid.h
    cy = grid.oy + (np.arange(grid.ny) + 0.5) * grid.h
    cz = grid.oz + (np.arange(grid.nz) + 0.5) * grid.h
    for x, y, z, p0, a in zip(*(np.asarray(balls[k], np.float64) for k in ("x", "y", "z", "p0", "a"))):
        if not a > 0:
            continue
        w = K * a if profile == GAUSS else a
        ii = np.nonzero(np.abs(cx - x) <= w)[0]
        jj = np.nonzero(np.abs(cy - y) <= w)[0]
        kk = np.nonzero(np.abs(cz - z) <= w)[0]
        if not (len(ii) and len(jj) and len(kk)):
            continue
        d2 = ((cx[ii] - x)[:, None, None] ** 2 + (cy[jj] - y)[None, :, None] ** 2
              + (cz[kk] - z)[None, None, :] ** 2)
        inside = d2 < w * w
        val = p0 * np.exp(-d2 / (2 * a * a)) if profile == GAUSS else np.full(d2.shape, p0)
        vol[np.ix_(ii, jj, kk)] += np.where(inside, val, 0.0)
    return vol


def gaussian_taps(sigma=1.5, radius=5):
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-t * t / (2 * sigma * sigma))
    return w / w.sum()


def _blur_valid(v, taps):
    for ax in range(3):
        v = np.apply_along_axis(lambda r: np.convolve(r, taps[::-1], mode="valid"), ax, v)
    return v


def metrics(img, ref, scale):
    """(MSE, PSNR dB, SSIM) of img against ref, both divided by scale."""
    x = np.asarray(img, np.float64) / scale
    y = np.asarray(ref, np.float64) / scale
    mse = float(np.mean((x - y) ** 2))
    psnr = 10.0 * np.log10(1.0 / mse) if mse > 0 else np.inf
    taps = gaussian_taps()
    mx, my = _blur_valid(x, taps), _blur_valid(y, taps)
    sx = _blur_valid(x * x, taps) - mx * mx
    sy = _blur_valid(y * y, taps) - my * my
    sxy = _blur_valid(x * y, taps) - mx * my
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    ssim = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))
    return mse, float(psnr), float(np.mean(ssim))
