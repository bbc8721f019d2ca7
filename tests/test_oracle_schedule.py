"""Pins of the oracle's composition of the schedule (oracle/schedule.py).

The paper fixes the schedule's structure but none of its constants (parity
unpinned, as for the growth thresholds), so these pins check that the
composition is what its steps make it: an empty stage changes nothing, a
filter-only stage is the zero-gradient filter, one iteration is one Adam step
on the masked parameters with the oracle's gradient, the softplus switch
leaves the forward model unchanged, and iterations lower the loss."""
import numpy as np
import pytest

import oracle
from oracle import schedule as osch
from paper_2601_00551_amd import synth


def _scene(seed=7, n_det=16, T=200):
    rng = np.random.default_rng(seed)
    arr = synth.hemisphere_array(n_det, 12.0, rng, tilt_deg=10.0)
    gt = synth.uniform_balls(rng, 60, 2.0, 0.15)
    init = synth.uniform_balls(rng, 120, 2.5, 0.15, 0.0, 0.2)
    base = oracle.Time(c=1.5, dt=0.05, T=T, f=1)
    return arr, gt, init, base, oracle.simulate(gt, arr, base)


def test_empty_stage_changes_nothing():
    arr, gt, init, base, y = _scene()
    cfg = osch.Config(base=base, stages=[osch.Stage(f=2, iters=0, filter=False)])
    st, recs = osch.run(init, arr, y, cfg)
    for k in oracle.PARAMS:
        np.testing.assert_array_equal(st.balls[k], np.asarray(init[k], np.float64))
    assert recs[0]["losses"] == [] and recs[0]["count_out"] == 120


def test_filter_stage_is_the_zero_gradient_filter():
    arr, gt, init, base, y = _scene()
    cfg = osch.Config(base=base, stages=[osch.Stage(f=2, iters=0, filter=True)])
    st, recs = osch.run(init, arr, y, cfg)
    keep, g, out = oracle.filter_zero_grad(init, arr, osch.level(base, 2), oracle.downsample(y, 2))
    assert recs[0]["count_filtered"] == keep.sum() == st.count()
    assert 0 < keep.sum() < 120
    np.testing.assert_array_equal(st.balls["x"], out["x"])


def test_one_iteration_is_one_adam_step_on_the_mask():
    arr, gt, init, base, y = _scene()
    cfg = osch.Config(base=base, stages=[osch.Stage(f=1, mask=osch.COARSE, iters=1, filter=False)])
    st, recs = osch.run(init, arr, y, cfg)
    b = {k: np.asarray(init[k], np.float64) for k in oracle.PARAMS}
    L, v = oracle.residual_loss(oracle.simulate(b, arr, base), y)
    g = oracle.vjp(b, arr, base, v)
    assert recs[0]["losses"] == [pytest.approx(L, rel=1e-14)]
    for i, k in enumerate(oracle.PARAMS):
        if k in osch.COARSE:
            n = len(b[k])
            want, _, _ = oracle.adam_step(b[k], g[k], np.zeros(n), np.zeros(n), 1, cfg.lr[i])
            np.testing.assert_allclose(st.balls[k], want, rtol=1e-14)
            # closed form of the first Adam step: -lr g / (|g| + eps)
            np.testing.assert_allclose(st.balls[k] - b[k], -cfg.lr[i] * g[k] / (np.abs(g[k]) + 1e-8),
                                       rtol=1e-9, atol=1e-15)
        else:
            np.testing.assert_array_equal(st.balls[k], b[k])


def test_softplus_switch_keeps_the_model():
    arr, gt, init, base, y = _scene()
    st = osch.State.start(init)
    L0, g0 = osch.loss_and_gradients(st, arr, base, y)
    osch.softplus_switch(st, True)
    L1, g1 = osch.loss_and_gradients(st, arr, base, y)
    assert L1 == pytest.approx(L0, rel=1e-12)
    # chain rule: dL/da~ = dL/da sigmoid(a~)
    np.testing.assert_allclose(g1["a"], g0["a"] * oracle.sigmoid(st.balls["a"]), rtol=1e-12)
    osch.softplus_switch(st, False)
    np.testing.assert_allclose(st.balls["a"], np.asarray(init["a"], np.float64), rtol=1e-12)


def test_two_level_schedule_lowers_the_loss():
    arr, gt, init, base, y = _scene()
    cfg = osch.Config(base=base, dup_frac=0.1, stages=[
        osch.Stage(f=2, mask=osch.COARSE, iters=8, grow_every=4),
        osch.Stage(f=1, mask=osch.ALL, iters=6, duplicate=True, softplus_frac=0.5)])
    st, recs = osch.run(init, arr, y, cfg)
    for r in recs:
        assert r["losses"][-1] < r["losses"][0]
    # the duplication at the change of rate adds balls to the filtered cloud
    assert recs[1]["count_entry"] > recs[1]["count_filtered"]
