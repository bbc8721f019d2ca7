"""The learned growth proposal end to end: training data from plain
reconstructions of four phantoms, training on the GPU, generalisation to the
candidates of two held-out phantoms (loss and ranking of the growth logit),
then the comparison with the plain method on two further phantoms (wall time
to the plain method's final residual).

Workload: the conformal array (512 elements on the jittered ellipsoid), a
branching-tree phantom, 2048 samples at 40 MHz with 5% noise, and a sparse
initial cloud of 20,000 lattice balls, where growth decides how fast the
phantom is covered.  The loss judge guarantees that every kept proposal
lowered the data-fidelity loss at its growth point."""
import json

import numpy as np
import pytest
import torch

from paper_2601_00551_amd import api, proposal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def _auc(score, label):
    """Area under the ROC curve (probability that a positive outranks a negative)."""
    order = np.argsort(score, kind="stable")
    ranks = np.empty(len(score))
    ranks[order] = np.arange(1, len(score) + 1)
    pos = label > 0.5
    n1, n0 = pos.sum(), (~pos).sum()
    return float((ranks[pos].sum() - n1 * (n1 + 1) / 2) / (n1 * n0))


def test_learned_proposal_gains_over_plain(ctx):
    grid = proposal.Grid.cube(10.0, 0.2)
    stages = proposal.default_schedule((4, 2, 1), iters=60)
    logs = []
    X, yg, yp = proposal.generate(ctx, range(4), grid, stages, n_init=20000,
                                  log=lambda s, **k: logs.append(s))
    assert len(X) == len(yg) == len(yp) > 0 and X.shape[1] == 31
    assert 0.0 < yg.mean() < 0.1
    # held-out phantoms: candidates of plain runs the network never sees
    Xh, ygh, yph = proposal.generate(ctx, range(4, 6), grid, stages, n_init=20000,
                                     log=lambda s, **k: logs.append(s))
    net = proposal.ProposalMLP(ctx, seed=0)
    dev = torch.device("cuda:0")
    probe = slice(0, min(len(Xh), 65536))
    as_dev = lambda a: torch.as_tensor(np.ascontiguousarray(a[probe], np.float32), device=dev)  # noqa: E731
    L_untrained = float(net.loss_and_grad(as_dev(Xh), as_dev(ygh), as_dev(yph), 1.0)[0].item())
    proposal.train(net, X, yg, yp, epochs=6, log=lambda s, **k: logs.append(s))
    L_trained = float(net.loss_and_grad(as_dev(Xh), as_dev(ygh), as_dev(yph), 1.0)[0].item())
    logit = net.forward(as_dev(Xh)).cpu().numpy()[:, 0]
    auc = _auc(logit, ygh[probe])
    print(json.dumps(dict(heldout_rows=int(len(Xh)), loss_untrained=L_untrained, loss_trained=L_trained,
                          auc=auc, positives=float(ygh.mean()))))
    # on the held-out phantoms: the loss falls well below the untrained
    # network's and the growth logit ranks growing sites above the others
    assert L_trained < 0.5 * L_untrained, (L_untrained, L_trained)
    assert auc > 0.75, auc
    rows = []
    for j in range(2):
        wl = proposal.proposal_workload(10_000 + j, n_init=20000)
        y = proposal.synthetic_measurement(ctx, wl, seed=60_000 + j)
        cap = 4 * len(wl.init["x"])
        _, plain = proposal.plain_run(ctx, wl, y, stages, capacity=cap)
        target = plain["final_loss"] * (1.0 + 1e-3)
        t_plain = proposal.first_below(plain["log"], target)
        lp = proposal.LearnedProposer(net, proposal.FeatureBuilder(ctx, grid, a_probe=0.1, half=10.0),
                                      a_init=wl.a_init, stages=[0])
        # same iteration mode as the plain run (eager), so the difference is the network's
        _, learned = proposal.plain_run(ctx, wl, y, stages, capacity=cap, stop_below=target, proposer=lp)
        for ev in lp.events:
            if ev["kept"]:
                assert ev["loss_after"] < ev["loss_before"], ev
        row = dict(phantom=10_000 + j, plain_s=t_plain, learned_s=learned["t_target"],
                   plain_final_loss=plain["final_loss"], kept=sum(e["kept"] for e in lp.events),
                   tried=len(lp.events))
        rows.append(row)
        print(json.dumps(row))
    for row in rows:
        assert row["learned_s"] is not None, row                  # reached the plain final residual
        assert row["learned_s"] < 1.1 * row["plain_s"], row       # never much later
    assert sum(r["learned_s"] for r in rows) < sum(r["plain_s"] for r in rows)   # and sooner overall
