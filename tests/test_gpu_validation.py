"""The binding rejects buffers shorter than the sizes passed beside them
(before any kernel runs), so a caller's mistake is a Python error, not a
GPU fault."""
import numpy as np
import pytest
import torch

from _util import PARAMS, gmodel, small_scene, to_dev
from paper_2601_00551_amd import api

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(gpu):
    ctx = api.Context(0)
    dev = torch.device("cuda:0")
    arr, balls = small_scene(501, nb=300, nd=7)
    yield ctx, dev, to_dev(arr, dev), to_dev(balls, dev)
    ctx.close()


def test_short_buffers_raise(setup):
    ctx, dev, A, B = setup
    T = 100
    m = gmodel(T)
    with pytest.raises(ValueError, match="y"):
        api.simulate_signals(ctx, A, B, m, y=torch.empty(1, 7, T - 1, device=dev))
    with pytest.raises(ValueError, match="balls"):
        api.simulate_signals(ctx, A, B, m, B_cap=301)
    with pytest.raises(ValueError, match="array"):
        api.simulate_signals(ctx, dict(A, nz=A["nz"][:6].contiguous()), B, m)
    with pytest.raises(ValueError, match="v"):
        api.adjoint_gradients(ctx, A, B, m, torch.zeros(7, T + 1, device=dev))
    with pytest.raises(ValueError, match="grad"):
        api.adjoint_gradients(ctx, A, B, m, torch.zeros(7, T, device=dev),
                              grad={k: torch.empty(299, device=dev) for k in PARAMS})
    y = torch.zeros(2, 7, T, device=dev)
    with pytest.raises(ValueError, match="out"):
        api.downsample(ctx, y, 4, out=torch.empty(2, 7, 24, device=dev))
    with pytest.raises(ValueError, match="out"):
        api.decimate(ctx, y, 3, out=torch.empty(2 * 7 * 33 + 1, device=dev))
    with pytest.raises(ValueError, match="f must"):
        api.decimate(ctx, y, 0)
    with pytest.raises(ValueError, match="y_ref"):
        api.residual_loss(ctx, y, torch.zeros(2, 7, T - 1, device=dev))
    with pytest.raises(ValueError, match="out"):
        api.filter_zero_grad(ctx, A, B, m, torch.zeros(1, 7, T, device=dev),
                             out={k: torch.empty(10, device=dev) for k in PARAMS})
    with pytest.raises(ValueError, match="y_ref"):
        api.filter_zero_grad(ctx, A, B, m, torch.zeros(1, 7, T - 1, device=dev))
    st = api.State({k: B[k].cpu().numpy() for k in PARAMS}, device=dev)
    with pytest.raises(ValueError, match="y_work"):
        api.step(ctx, A, st, m, torch.zeros(1, 7, T, device=dev), torch.empty(1, 7, T - 1, device=dev),
                 api.AdamParams())


def test_exact_buffers_still_run(setup):
    ctx, dev, A, B = setup
    T = 100
    y = api.simulate_signals(ctx, A, B, gmodel(T), y=torch.empty(1, 7, T, device=dev))
    g = api.adjoint_gradients(ctx, A, B, gmodel(T), y)
    assert all(torch.isfinite(g[k]).all() for k in PARAMS)
    assert api.decimate(ctx, y, 3).shape == (1, 7, 33)


def test_image_and_proposal_buffers(setup):
    from paper_2601_00551_amd import envelope, image, proposal
    ctx, dev, A, B = setup
    grid = proposal.Grid.cube(2.0, 0.5)
    off = torch.tensor([0, B["x"].numel()], dtype=torch.int64, device=dev)
    with pytest.raises(ValueError, match="vox"):
        image.voxelize(ctx, B, off, api.Model(), grid, vox=torch.empty(grid.ncell - 1, device=dev))
    n = grid.ncell
    img = torch.zeros(n, device=dev)
    with pytest.raises(ValueError, match="work"):
        image.metrics(ctx, img, img, (grid.nx, grid.ny, grid.nz), 1.0, work=torch.empty(10 * n - 1, device=dev))
    with pytest.raises(ValueError, match="mass"):
        proposal.grid_mass(ctx, B, off, grid, mass=torch.empty(n + 1, device=dev))
    tri = torch.zeros(9, device=dev)
    x = torch.zeros(5, device=dev)
    with pytest.raises(ValueError, match="y"):
        envelope.mesh_inside(ctx, tri, x, torch.zeros(4, device=dev), x)
    mlp = proposal.ProposalMLP(ctx)
    X = torch.zeros(10, proposal.MLP_IN, device=dev)
    with pytest.raises(ValueError, match="out"):
        mlp.forward(X, out=torch.empty(10, 1, device=dev))
    assert mlp.forward(X).shape == (10, 2)
