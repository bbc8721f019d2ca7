"""The learned growth proposal end to end on small conformal workloads:
training data from plain reconstructions, training on the GPU, then the
comparison with the plain method on a held-out phantom (wall time to the
plain method's final residual).  The loss judge guarantees that every kept
proposal lowered the data-fidelity loss at its growth point."""
import json

import numpy as np
import pytest
import torch

from paper_2601_00551_amd import api, proposal, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def small_workload(index, n_init=20000, n_det=128):
    rng = synth.rng_for(5, 500 + index)
    arr = synth.ellipsoid_array(n_det, (20.0, 15.0, 10.0), rng, jitter=1.0)
    region = synth.Region(10.0, (18.0, 13.0, 8.0))
    gt = synth.drop_near(synth.tree_phantom(rng, region, max_depth=4), arr, 1.5)
    init = synth.drop_near(synth.region_init(rng, region, n_init), arr, 1.5)
    return synth.Workload(f"small-proposal-{index}", arr, gt, init, 1024, 0.025, (4, 2, 1), 0.1)


def test_learned_proposal_against_plain(ctx):
    grid = proposal.Grid.cube(10.0, 0.2)
    stages = proposal.default_schedule((4, 2, 1), iters=30, grow_every=10)
    logs = []
    X, yg, yp = proposal.generate(ctx, range(3), grid, stages, workload=small_workload,
                                  log=lambda s, **k: logs.append(s))
    assert len(X) == len(yg) == len(yp) > 0 and X.shape[1] == 31
    assert 0.0 < yg.mean() < 1.0
    net = proposal.ProposalMLP(ctx, seed=1)
    hist = proposal.train(net, X, yg, yp, epochs=4, batch=4096, lr=1e-3, log=lambda s, **k: logs.append(s))
    assert hist[-1] < hist[0]
    wl = small_workload(100)
    y = proposal.synthetic_measurement(ctx, wl, seed=7)
    cap = 4 * len(wl.init["x"])
    _, plain = proposal.plain_run(ctx, wl, y, stages, capacity=cap)
    lp = proposal.LearnedProposer(net, proposal.FeatureBuilder(ctx, grid, a_probe=0.1, half=10.0),
                                  a_init=wl.a_init)
    _, learned = proposal.plain_run(ctx, wl, y, stages, capacity=cap, stop_below=plain["final_loss"],
                                    proposer=lp)
    assert lp.events, "no growth point was reached"
    for ev in lp.events:
        if ev["kept"]:
            assert ev["loss_after"] < ev["loss_before"], ev
    row = dict(plain_wall_s=plain["wall_s"], plain_final_loss=plain["final_loss"],
               learned_t_target=learned["t_target"], learned_wall_s=learned["wall_s"],
               learned_final_loss=learned["final_loss"], kept=sum(e["kept"] for e in lp.events),
               tried=len(lp.events), accepted=[e["accepted"] for e in lp.events])
    print(json.dumps(row))
    assert np.isfinite(learned["final_loss"])
