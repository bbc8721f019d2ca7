"""Pins of the voxelisation and image-quality reference (no GPU): closed forms
of a single ball, the Gaussian's integral, linearity, and the SSIM / PSNR
values of images whose answer is known."""
import numpy as np
import pytest

from oracle import image as oi
from oracle.proposal import Grid


def _ball(x, y, z, p0, a):
    return {"x": np.array([x]), "y": np.array([y]), "z": np.array([z]), "p0": np.array([p0]), "a": np.array([a])}


def test_single_gaussian_ball_values():
    g = Grid(-1.0, -1.0, -1.0, 0.1, 20, 20, 20)
    # centre of voxel (10, 10, 10) is (0.05, 0.05, 0.05)
    v = oi.voxelize(_ball(0.05, 0.05, 0.05, 0.8, 0.12), g)
    assert v[10, 10, 10] == pytest.approx(0.8, rel=1e-15)
    assert v[11, 10, 10] == pytest.approx(0.8 * np.exp(-0.01 / (2 * 0.0144)), rel=1e-12)
    assert v[11, 11, 9] == pytest.approx(0.8 * np.exp(-0.03 / (2 * 0.0144)), rel=1e-12)
    # truncation at K a = 0.6: a voxel 0.7 away is empty, one 0.5 away is not
    assert v[17, 10, 10] == 0.0 and v[15, 10, 10] > 0.0


def test_gaussian_integral():
    """sum(vox) h^3 -> p0 (2 pi a^2)^(3/2) for a ball well resolved by the grid."""
    g = Grid(-2.0, -2.0, -2.0, 0.05, 80, 80, 80)
    a = 0.3
    v = oi.voxelize(_ball(0.013, -0.021, 0.007, 1.0, a), g, K=6.0)
    assert v.sum() * 0.05 ** 3 == pytest.approx((2 * np.pi * a * a) ** 1.5, rel=1e-6)


def test_uniform_ball_counts_voxels_inside():
    g = Grid(-1.0, -1.0, -1.0, 0.1, 20, 20, 20)
    v = oi.voxelize(_ball(0.0, 0.0, 0.0, 2.0, 0.35), g, profile=oi.UNIFORM)
    c = -1.0 + (np.arange(20) + 0.5) * 0.1
    d2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    np.testing.assert_array_equal(v, np.where(d2 < 0.35 ** 2, 2.0, 0.0))


def test_linearity_and_dead_balls():
    g = Grid(-1.0, -1.0, -1.0, 0.1, 20, 20, 20)
    b1, b2 = _ball(0.1, 0.2, -0.1, 0.5, 0.1), _ball(-0.3, 0.0, 0.2, 0.7, 0.15)
    both = {k: np.concatenate([b1[k], b2[k]]) for k in b1}
    np.testing.assert_allclose(oi.voxelize(both, g), oi.voxelize(b1, g) + oi.voxelize(b2, g), rtol=1e-15)
    assert np.all(oi.voxelize(_ball(0.0, 0.0, 0.0, 1.0, -0.1), g) == 0.0)


def test_taps():
    w = oi.gaussian_taps()
    assert len(w) == 11 and w.sum() == pytest.approx(1.0, abs=1e-15)
    assert w[5] / w[6] == pytest.approx(np.exp(1 / (2 * 2.25)))


def test_ssim_identity_and_constants():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(14, 13, 12))
    mse, psnr, ssim = oi.metrics(x, x, 1.0)
    assert mse == 0.0 and psnr == np.inf and ssim == pytest.approx(1.0, abs=1e-12)
    # constant volumes alpha, beta: SSIM = (2 ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    mse, psnr, ssim = oi.metrics(np.full((12, 12, 12), a), np.full((12, 12, 12), b), 1.0)
    C1 = 1e-4
    assert ssim == pytest.approx((2 * a * b + C1) / (a * a + b * b + C1), rel=1e-10)
    assert mse == pytest.approx(0.16) and psnr == pytest.approx(10 * np.log10(1 / 0.16))


def test_ssim_contrast_and_scale():
    """y = 2 x with zero-mean x: means vanish, so SSIM = (2*2 sxx + C2)/(5 sxx + C2)
    wherever the local variance is uniform (here: a +-d checkerboard)."""
    i, j, k = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    d = 0.1
    x = np.where((i + j + k) % 2 == 0, d, -d)
    _, _, s = oi.metrics(x, 2 * x, 1.0)
    taps = oi.gaussian_taps()
    # local mean of the checkerboard and of its square, in the 'valid' interior
    mx = np.prod([np.sum(taps * np.where(np.arange(11) % 2 == 0, 1, -1)) for _ in range(3)]) * d
    sxx = d * d - mx * mx
    C1, C2 = 1e-4, 9e-4
    exp_ = ((2 * mx * 2 * mx + C1) * (2 * 2 * sxx + C2)) / ((mx * mx + 4 * mx * mx + C1) * (5 * sxx + C2))
    # the sign of mx alternates from voxel to voxel but enters squared or paired
    assert s == pytest.approx(exp_, rel=1e-9)
    # dividing both volumes by the same scale is the normalisation
    m1 = oi.metrics(3 * x, 6 * x, 3.0)
    assert m1[2] == pytest.approx(s, rel=1e-12)
