"""The learned proposal's gate (host logic, no GPU): the network is used only
while the loss judge keeps what it proposes."""
import torch

from paper_2601_00551_amd import proposal


class Scripted(proposal.LearnedProposer):
    """A proposer whose proposals the judge keeps or rejects by script."""

    def __init__(self, verdicts, **kw):
        super().__init__(mlp=None, builder=None, **kw)
        self.verdicts = list(verdicts)
        self.calls = 0

    def _propose(self, r, model, y_k, yw, ev):
        self.calls += 1
        ev["kept"] = self.verdicts.pop(0)


def _call(p, stage=0):
    p(None, stage, None, None, torch.zeros(1))


def test_gate_closes_after_patience_rejections_in_a_row():
    p = Scripted([False, True, False, False, True], patience=2)
    p.new_run()
    for _ in range(5):
        _call(p)
    # reject, keep (resets), reject, reject -> closed; the fifth call is skipped
    assert p.calls == 4 and p.gated
    assert [e.get("gate_closed", False) for e in p.events] == [False, False, False, True]


def test_per_run_gate_reopens_each_run():
    p = Scripted([False, False, True], patience=1)
    p.new_run()
    _call(p), _call(p)
    assert p.calls == 1 and p.gated
    p.new_run()
    assert not p.gated
    _call(p)
    assert p.calls == 2


def test_gate_carried_over_runs_reprobes_every_n_runs():
    p = Scripted([False] * 10, patience=1, reprobe_every=3)
    tried = []
    for run in range(1, 9):
        p.new_run()
        before = p.calls
        _call(p), _call(p)
        tried.append(p.calls - before)
    # run 1 probes and closes; reopened for one probe in runs 4 and 7
    assert tried == [1, 0, 0, 1, 0, 0, 1, 0]
    assert [e["run"] for e in p.events] == [1, 4, 7]


def test_no_patience_never_closes_and_stages_filter():
    p = Scripted([False] * 4, patience=None, stages=[0])
    p.new_run()
    for _ in range(3):
        _call(p)
    _call(p, stage=1)          # not a stage it acts in
    assert p.calls == 3 and not p.gated


def test_max_per_stage_counts_this_run_only():
    p = Scripted([True] * 6, max_per_stage=1)
    p.new_run()
    _call(p), _call(p)
    p.new_run()
    _call(p)
    assert p.calls == 2
