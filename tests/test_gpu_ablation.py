"""The Pro-vs-SlingBAG-style comparison end to end on a small conformal
workload: both schedules run, the quality probe records finite figures, the
filter shrinks Pro's cloud, and the probe's measuring time is excluded from
the reported wall times (behavioural checks; the figures themselves are
measurements, not parity)."""
import numpy as np
import pytest
import torch

from paper_2601_00551_amd import ablation, api, image, proposal, synth

pytestmark = pytest.mark.gpu


def test_pro_and_slingbag_schedules_run_and_are_probed(gpu):
    ctx = api.Context(0)
    rng = synth.rng_for(2, 300)
    arr = synth.ellipsoid_array(128, (20.0, 15.0, 10.0), rng, jitter=1.0)
    region = synth.Region(10.0, (18.0, 13.0, 8.0))
    gt = synth.drop_near(synth.tree_phantom(rng, region, max_depth=4), arr, 1.5)
    init = synth.drop_near(synth.region_init(rng, region, 20000), arr, 1.5)
    wl = synth.Workload("small", arr, gt, init, 1024, 0.025, (4, 2, 1), 0.1)
    ys = {smp: proposal.synthetic_measurement(ctx, wl, seed=9, sampling=smp)
          for smp in (api.SAMPLING_BIN, api.SAMPLING_POINT)}
    grid = proposal.Grid.cube(10.0, 0.4)
    dev = torch.device("cuda:0")
    g = {k: torch.as_tensor(np.asarray(v), device=dev) for k, v in wl.gt.items()}
    gt_vol = image.voxelize(ctx, g, torch.tensor([0, len(wl.gt["x"])], device=dev), api.Model(), grid)
    res = {}
    for name, (sched, smp) in ablation.VARIANTS.items():
        res[name] = ablation.run(ctx, wl, ys[smp], sched(iters=20), grid, gt_vol, every=5,
                                 capacity=4 * len(init["x"]), sampling=smp)
        tr = res[name]["trace"]
        assert len(tr) >= 3
        assert all(np.isfinite(r["psnr"]) and -1.0 <= r["ssim"] <= 1.0 for r in tr)
        assert all(b["t"] >= a["t"] for a, b in zip(tr, tr[1:]))
        assert 0.0 < res[name]["wall_s"] <= tr[-1]["t"] + 1e-3
    # the zero-gradient filter removes balls at Pro's first stage entry
    assert res["pro"]["trace"][0]["balls"] < len(init["x"])
    assert res["pro_point"]["trace"][0]["balls"] < len(init["x"])
    ctx.close()
