"""The hierarchical driver end to end on small synthetic workloads: the loss
falls in every stage, graph-captured iterations track eager ones, and a run
interrupted by an injected failure resumes from its checkpoint to the same
result.  (The schedule and thresholds are readings of the paper, so these are
behavioural checks, not oracle parity.)"""
import numpy as np
import pytest
import torch

from paper_2601_00551_amd import api, recon, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def measured(ctx, wl, noise=0.0, seed=0):
    dev = torch.device("cuda:0")
    A = {k: torch.as_tensor(v, device=dev) for k, v in wl.array.items()}
    gt = {k: torch.as_tensor(v, device=dev) for k, v in wl.gt.items()}
    m = api.Model(c=1.5, dt=wl.dt, T=wl.T, f=1)
    y = api.simulate_signals(ctx, A, gt, m)
    if noise > 0:
        rng = np.random.default_rng(seed)
        sigma = noise * float(y.abs().max())
        y = y + sigma * torch.as_tensor(rng.normal(size=tuple(y.shape)).astype(np.float32), device=dev)
    return y.contiguous()


def small_conformal(seed=0, n_det=128, n_init=20000):
    rng = synth.rng_for(2, 100 + seed)
    arr = synth.ellipsoid_array(n_det, (20.0, 15.0, 10.0), rng, jitter=1.0)
    region = synth.Region(10.0, (18.0, 13.0, 8.0))
    gt = synth.drop_near(synth.tree_phantom(rng, region, max_depth=4), arr, 1.5)
    init = synth.drop_near(synth.region_init(rng, region, n_init), arr, 1.5)
    return synth.Workload("small-conformal", arr, gt, init, 1024, 0.025, (4, 2, 1), 0.1)


def test_tiny_plain_reconstruction_converges(ctx):
    wl = synth.tiny_config()
    y = measured(ctx, wl)
    cfg = recon.ReconConfig(stages=[recon.Stage(f=1, mask=api.COARSE, iters=50, filter=True, tol=0.0)],
                            T=wl.T, dt=wl.dt)
    r = recon.Recon(wl.array, y, wl.init, cfg, ctx=ctx)
    out = r.run()
    losses = [e["loss"] for e in out["log"] if e["kind"] == "iter"]
    assert len(losses) == 50
    # positions stay on the 0.625 mm lattice in the coarse stage: a partial fit
    assert losses[-1] < 0.4 * losses[0]
    assert np.mean(losses[-10:]) < np.mean(losses[:10])
    n = out["state"].count()
    assert 0 < n <= len(wl.init["x"])


def test_three_level_schedule(ctx):
    wl = small_conformal()
    y = measured(ctx, wl, noise=0.05)
    stages = recon.plain_schedule((4, 2, 1), iters=30, coarse_grow_every=10, fine_grow_every=10,
                                  softplus_frac=0.2, tol=0.0)
    cfg = recon.ReconConfig(stages=stages, T=wl.T, dt=wl.dt, dup_frac=0.05)
    out = recon.Recon(wl.array, y, wl.init, cfg, ctx=ctx).run()
    log = out["log"]
    for si in range(3):
        it = [e["loss"] for e in log if e["stage"] == si and e["kind"] == "iter"]
        assert len(it) == 30 and it[-1] < it[0], si
    st = out["state"]
    n = st.count()
    a = st.balls["a"][:n].cpu().numpy()
    assert n > 0 and np.all(a > 0)
    entries = [e for e in log if e["kind"] == "stage-entry"]
    assert [e["f"] for e in entries] == [4, 2, 1]


def test_graph_mode_tracks_eager(ctx):
    wl = small_conformal(seed=1, n_init=8000)
    y = measured(ctx, wl)
    mk = lambda gi: recon.ReconConfig(stages=[recon.Stage(f=2, mask=api.ALL, iters=20, filter=True,
                                                          grow_every=10, tol=0.0)],
                                      T=wl.T, dt=wl.dt, graph_iters=gi)
    a = recon.Recon(wl.array, y, wl.init, mk(0), ctx=ctx).run()
    b = recon.Recon(wl.array, y, wl.init, mk(5), ctx=ctx).run()
    la = [e["loss"] for e in a["log"] if e["kind"] == "iter"]
    lb = [e["loss"] for e in b["log"] if e["kind"] == "iter"]
    assert len(la) == len(lb) == 20
    np.testing.assert_allclose(lb, la, rtol=2e-3)


def test_checkpoint_resume_after_injected_failure(ctx, tmp_path):
    wl = small_conformal(seed=2, n_init=8000)
    y = measured(ctx, wl)
    stages = recon.plain_schedule((4, 2), iters=16, coarse_grow_every=8, fine_grow_every=8,
                                  softplus_frac=0.25, tol=0.0)

    def cfg(d):
        return recon.ReconConfig(stages=stages, T=wl.T, dt=wl.dt, checkpoint_dir=str(d),
                                 checkpoint_every=4, dup_frac=0.05)
    full = recon.Recon(wl.array, y, wl.init, cfg(tmp_path / "a"), ctx=ctx).run()
    with pytest.raises(recon.InjectedFailure):
        recon.Recon(wl.array, y, wl.init, cfg(tmp_path / "b"), ctx=ctx).run(fail_at=(1, 14))
    resumed = recon.Recon(wl.array, y, wl.init, cfg(tmp_path / "b"), ctx=ctx).run(resume=True)
    na, nb = full["state"].count(), resumed["state"].count()
    assert na == nb
    assert resumed["final_loss"] == pytest.approx(full["final_loss"], rel=1e-3)
    for k in api.PARAMS:
        a = full["state"].balls[k][:na].cpu().numpy()
        b = resumed["state"].balls[k][:nb].cpu().numpy()
        assert np.max(np.abs(a - b)) <= 1e-3 * max(1.0, np.abs(a).max()), k
