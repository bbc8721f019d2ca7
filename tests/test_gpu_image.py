"""GPU parity of the voxelisation and image-quality kernels against the FP64
reference (oracle/image.py), through the C-ABI.

Tolerances: voxels are FP32 sums of FP32 exponentials (relative 1e-5 of the
volume's maximum); MSE relative 1e-5; PSNR 1e-4 dB; SSIM 2e-5 absolute (FP32
separable blur of five fields, 1331 taps per voxel)."""
import numpy as np
import pytest
import torch

from oracle import image as oi
from oracle.proposal import Grid as OGrid
from paper_2601_00551_amd import api, image, proposal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def _cloud(rng, n, half, a_lo=0.06, a_hi=0.25):
    b = {k: rng.uniform(-half, half, n).astype(np.float32) for k in ("x", "y", "z")}
    b["p0"] = rng.uniform(-0.2, 1.0, n).astype(np.float32)
    b["a"] = rng.uniform(a_lo, a_hi, n).astype(np.float32)
    b["a"][:5] = -0.1     # dead balls
    return b


def _dev(b):
    return {k: torch.as_tensor(v, device="cuda:0") for k, v in b.items()}


@pytest.mark.parametrize("profile", [api.PROFILE_GAUSS, api.PROFILE_UNIFORM])
def test_voxelize_matches_oracle(ctx, profile):
    rng = np.random.default_rng(10 + profile)
    b = _cloud(rng, 1500, 1.3)
    g = proposal.Grid(-1.5, -1.4, -1.2, 0.1, 30, 28, 25)
    off = torch.tensor([0, 1500], dtype=torch.int64, device="cuda:0")
    m = api.Model(profile=profile, gauss_K=5.0)
    v = image.voxelize(ctx, _dev(b), off, m, g).cpu().numpy().reshape(30, 28, 25)
    ref = oi.voxelize(b, OGrid(g.ox, g.oy, g.oz, g.h, g.nx, g.ny, g.nz), profile=profile, K=5.0)
    assert np.max(np.abs(v - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_voxelize_softplus_sizes_and_frame_range(ctx):
    rng = np.random.default_rng(3)
    b = _cloud(rng, 800, 1.0)
    g = proposal.Grid(-1.2, -1.2, -1.2, 0.08, 30, 30, 30)
    og = OGrid(g.ox, g.oy, g.oz, g.h, g.nx, g.ny, g.nz)
    at = np.log(np.expm1(np.abs(b["a"]).astype(np.float64))).astype(np.float32)   # a~ with softplus(a~) = |a|
    bs = dict(b, a=at)
    off = torch.tensor([100, 700], dtype=torch.int64, device="cuda:0")
    v = image.voxelize(ctx, _dev(bs), off, api.Model(a_softplus=1), g).cpu().numpy().reshape(30, 30, 30)
    sub = {k: np.asarray(x)[100:700] for k, x in b.items()}
    sub["a"] = np.abs(sub["a"])
    ref = oi.voxelize(sub, og)
    assert np.max(np.abs(v - ref)) <= 2e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(11, 11, 11), (23, 17, 13), (40, 36, 32)])
def test_metrics_match_oracle(ctx, shape):
    rng = np.random.default_rng(sum(shape))
    n = int(np.prod(shape))
    ref = rng.uniform(0, 1, size=shape).astype(np.float32)
    ref = np.where(rng.uniform(size=shape) < 0.8, 0.0, ref).astype(np.float32)
    img = (ref + 0.1 * rng.normal(size=shape)).astype(np.float32)
    scale = float(ref.max())
    out = image.metrics(ctx, torch.as_tensor(img.ravel(), device="cuda:0"),
                        torch.as_tensor(ref.ravel(), device="cuda:0"), shape, scale).cpu().numpy()
    mse, psnr, ssim = oi.metrics(img, ref, scale)
    assert out[0] == pytest.approx(mse, rel=1e-5)
    assert out[1] == pytest.approx(psnr, abs=1e-4)
    assert out[2] == pytest.approx(ssim, abs=2e-5)


def test_metrics_identical_volumes(ctx):
    rng = np.random.default_rng(5)
    x = torch.as_tensor(rng.uniform(size=12 * 13 * 14).astype(np.float32), device="cuda:0")
    out = image.metrics(ctx, x, x, (12, 13, 14), 1.0).cpu().numpy()
    assert out[0] == 0.0 and np.isinf(out[1]) and out[2] == pytest.approx(1.0, abs=1e-6)


def test_reconstruction_quality_pipeline(ctx):
    """Voxelised ground truth against a perturbed copy: the figures follow the
    reference computed from the oracle's own voxelisation."""
    rng = np.random.default_rng(8)
    gt = _cloud(rng, 3000, 1.8, 0.08, 0.12)
    gt["p0"] = np.abs(gt["p0"]).astype(np.float32)
    gt["a"] = np.abs(gt["a"]).astype(np.float32)
    rec = {k: v.copy() for k, v in gt.items()}
    rec["x"] += rng.normal(0, 0.03, 3000).astype(np.float32)
    rec["p0"] *= rng.uniform(0.8, 1.2, 3000).astype(np.float32)
    g = proposal.Grid(-2.0, -2.0, -2.0, 0.1, 40, 40, 40)
    og = OGrid(g.ox, g.oy, g.oz, g.h, g.nx, g.ny, g.nz)
    off = torch.tensor([0, 3000], dtype=torch.int64, device="cuda:0")
    m = api.Model()
    vg = image.voxelize(ctx, _dev(gt), off, m, g)
    vr = image.voxelize(ctx, _dev(rec), off, m, g)
    scale = float(vg.max())
    out = image.metrics(ctx, vr, vg, (40, 40, 40), scale).cpu().numpy()
    ref = oi.metrics(oi.voxelize(rec, og), oi.voxelize(gt, og), scale)
    assert out[1] == pytest.approx(ref[1], abs=1e-3)
    assert out[2] == pytest.approx(ref[2], abs=1e-4)
