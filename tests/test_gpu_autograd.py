"""The autograd binding: gradients through SimulateFn agree with the oracle's
dual-number gradients (FP32) and pass torch.autograd.gradcheck (FP64 twins)."""
import numpy as np
import pytest
import torch

import oracle
from _util import PARAMS, gmodel, otime, rel_l2, small_scene, to_dev
from paper_2601_00551_amd import api
from paper_2601_00551_amd.autograd import simulate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def test_loss_backward_matches_oracle(ctx):
    dev = torch.device("cuda:0")
    arr, balls = small_scene(201, nb=1800, nd=23)
    T = 450
    rng = np.random.default_rng(1)
    gt = dict(balls, p0=(balls["p0"] * rng.uniform(0.5, 1.5, len(balls["p0"]))).astype(np.float32))
    y_ref = oracle.simulate(gt, arr, otime(T)).astype(np.float32)
    t = {k: torch.tensor(balls[k], device=dev, requires_grad=True) for k in PARAMS}
    y = simulate(t["x"], t["y"], t["z"], t["p0"], t["a"], to_dev(arr, dev), gmodel(T), sbp_ctx=ctx)
    loss = ((y[0] - torch.as_tensor(y_ref, device=dev)) ** 2).sum()
    loss.backward()
    ys = oracle.simulate(balls, arr, otime(T))
    L, v = oracle.residual_loss(ys, y_ref)
    ref = oracle.vjp(balls, arr, otime(T), v)
    assert loss.item() == pytest.approx(L, rel=1e-5)
    for k in PARAMS:
        assert rel_l2(t[k].grad.cpu().numpy(), ref[k]) <= 1e-4, k


def test_partial_requires_grad(ctx):
    dev = torch.device("cuda:0")
    arr, balls = small_scene(202, nb=300, nd=7)
    T = 450
    t = {k: torch.tensor(balls[k], device=dev, requires_grad=(k in ("p0", "a"))) for k in PARAMS}
    y = simulate(t["x"], t["y"], t["z"], t["p0"], t["a"], to_dev(arr, dev), gmodel(T), sbp_ctx=ctx)
    (y ** 2).sum().backward()
    assert t["x"].grad is None and t["p0"].grad is not None and t["a"].grad is not None


@pytest.mark.parametrize("sampling", [api.SAMPLING_BIN, api.SAMPLING_POINT])
def test_gradcheck_fp64(ctx, sampling):
    """Central finite differences of the FP64 GPU forward against its FP64 adjoint,
    for bin means and point samples."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(203)
    arr, balls = small_scene(203, nb=6, nd=5, radius=9.0, half=1.5)
    T = 500
    A = to_dev(arr, dev, torch.float64)
    t = [torch.tensor(balls[k], dtype=torch.float64, device=dev, requires_grad=True) for k in PARAMS]
    w = torch.as_tensor(rng.normal(size=(1, 5, T)), device=dev)
    fn = lambda *p: (simulate(*p, A, gmodel(T, sampling=sampling), sbp_ctx=ctx) * w).sum()
    assert torch.autograd.gradcheck(fn, tuple(t), eps=1e-6, atol=1e-7, rtol=1e-5)


@pytest.mark.slow
def test_large_subset_fd_fp64(ctx):
    """The large workload's transducer cap with the first 1,000 balls of its
    cloud: FP64 GPU gradients vs central finite differences of the FP64 GPU
    forward for a sample of balls and every parameter, and vs the oracle."""
    from paper_2601_00551_amd import synth
    dev = torch.device("cuda:0")
    wl = synth.large_config(n_balls=1000)
    T = 4096
    balls = wl.init
    A = to_dev(wl.array, dev, torch.float64)
    m = gmodel(T)
    rng = np.random.default_rng(3)
    v = torch.as_tensor(rng.normal(size=(1, len(wl.array["qx"]), T)), device=dev)
    t = {k: torch.tensor(balls[k], dtype=torch.float64, device=dev, requires_grad=True) for k in PARAMS}
    y = simulate(t["x"], t["y"], t["z"], t["p0"], t["a"], A, m, sbp_ctx=ctx)
    (y * v).sum().backward()
    sample = rng.choice(1000, size=12, replace=False)
    for k in PARAMS:
        h = 1e-6 if k in ("x", "y", "z") else 1e-6 * float(np.abs(balls[k]).mean())
        for i in sample:
            # the signal is a sum over balls, so the loss's derivative in ball i's
            # parameter is that of ball i's own term: difference one ball alone
            one = {kk: torch.tensor(balls[kk][i:i + 1], dtype=torch.float64, device=dev) for kk in PARAMS}
            bp = {kk: vv.clone() for kk, vv in one.items()}
            bm = {kk: vv.clone() for kk, vv in one.items()}
            bp[k][0] += h
            bm[k][0] -= h
            fp = (api.simulate_signals_f64(ctx, A, bp, m) * v).sum().item()
            fm = (api.simulate_signals_f64(ctx, A, bm, m) * v).sum().item()
            fd = (fp - fm) / (2 * h)
            g = t[k].grad[i].item()
            assert abs(g - fd) <= 1e-5 * max(abs(fd), 1e-3 * float(t[k].grad.abs().max())), (k, i, g, fd)
    ref = oracle.vjp(balls, wl.array, otime(T), v[0].cpu().numpy(), ball_idx=sample)
    for k in PARAMS:
        assert rel_l2(t[k].grad[sample].cpu().numpy(), ref[k]) <= 1e-9, k
