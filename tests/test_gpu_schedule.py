"""The schedule driver (Algorithm 1, paper_2601_00551_amd/recon.py) against the
oracle's composition of the same steps (oracle/schedule.py), on a tiny
two-level run: coarse stage at half rate (p0 and a, split / destroy after
three iterations), fine stage at full rate (filter, duplication at the change
of rate, all five parameters, the last 40 % on a~ with a = softplus(a~)).

Step by step: every call the driver makes is recorded with the state before
and after it, the oracle applies the same step to the recorded state before,
and the result is compared with the recorded state after -- Downsample_f,
the zero-gradient filter (keep-set equal outside the 1e-6 band, moments
carried), the duplication gradients and the growth rule (counts, order,
positions, zero moments for new balls), every iteration (loss, the masked
gradients, Adam with the stage's mask, learning rates and a step count that
restarts at every stage, the unmasked parameters untouched) and the softplus
switches.  Then an independent FP64 run of the whole schedule from the same
start: the same ball counts at every stage boundary and per-iteration losses
within 1e-3."""
import numpy as np
import pytest
import torch

import oracle
from oracle import schedule as osch
from _util import rel_l2
from paper_2601_00551_amd import api, recon, synth

pytestmark = pytest.mark.gpu

T, DT = 256, 0.05
LR = (0.005, 0.005, 0.005, 0.02, 0.002)
GROWTH = dict(destroy_frac=0.02, a_min=0.02, a_split=0.1535, dup_offset=0.5)
DUP = 0.1


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def scene():
    rng = np.random.default_rng(2026)
    arr = synth.hemisphere_array(24, 15.0, rng, tilt_deg=10.0)
    gt = synth.polyline_phantom(rng, per_line=100)
    init = synth.cube_lattice(8, 5.0, 0.15)
    init["p0"] = rng.uniform(0.0, 0.2, len(init["x"])).astype(np.float32)
    base = oracle.Time(c=1.5, dt=DT, T=T, f=1, profile=oracle.GAUSS, directivity=oracle.COS)
    y_real = oracle.simulate(gt, arr, base).astype(np.float32)
    return arr, init, y_real, base


def snap(st):
    n = st.count()
    return {name: {k: getattr(st, name)[k][:n].detach().cpu().numpy().astype(np.float64) for k in api.PARAMS}
            for name in ("balls", "grad", "m", "v")}


def o_state(s, softplus=False):
    return osch.State({k: v.copy() for k, v in s["balls"].items()}, {k: v.copy() for k, v in s["grad"].items()},
                      {k: v.copy() for k, v in s["m"].items()}, {k: v.copy() for k, v in s["v"].items()}, softplus)


def otime(model):
    return oracle.Time(c=model.c, dt=model.dt, t0=model.t0, T=model.T, f=model.f, profile=oracle.GAUSS,
                       directivity=oracle.COS, K=model.gauss_K)


def kept_mask(before, after):
    """Which balls of `before` the order-preserving compaction kept (exact copies)."""
    bx, ax = before["balls"], after["balls"]
    keep = np.zeros(len(bx["x"]), dtype=bool)
    j = 0
    for i in range(len(bx["x"])):
        if j < len(ax["x"]) and all(bx[k][i] == ax[k][j] for k in ("x", "y", "z", "a", "p0")):
            keep[i] = True
            j += 1
    assert j == len(ax["x"])
    return keep


@pytest.fixture(scope="module")
def run(ctx, request):
    arr, init, y_real, base = scene()
    dev = torch.device("cuda:0")
    cfg = recon.ReconConfig(
        stages=[recon.Stage(f=2, mask=api.COARSE, iters=6, filter=True, grow_every=3, tol=0.0),
                recon.Stage(f=1, mask=api.ALL, iters=5, filter=True, duplicate=True, tol=0.0,
                            softplus_frac=0.4)],
        T=T, dt=DT, tuning=None, lr=LR, growth=dict(GROWTH), dup_frac=DUP, capacity=4 * len(init["x"]))
    r = recon.Recon(arr, torch.as_tensor(y_real, device=dev), init, cfg, ctx=ctx)
    ev = []
    mp = pytest.MonkeyPatch()
    request.addfinalizer(mp.undo)

    def wrap_method(name, kind):
        orig = getattr(r, name)

        def w(*a, **k):
            before = snap(r.state)
            out = orig(*a, **k)
            torch.cuda.synchronize()
            ev.append((kind, before, snap(r.state), a))
            return out
        setattr(r, name, w)

    wrap_method("_filter", "filter")
    wrap_method("_gradients", "gradients")
    wrap_method("_grow", "grow")
    orig_step, orig_rep, orig_ds = api.step, api.softplus_reparam, api.downsample

    def step(ctx_, A, st, model, y_k, yw, prm, loss=None, stream=None):
        before = snap(st)
        out = orig_step(ctx_, A, st, model, y_k, yw, prm, loss=loss, stream=stream)
        torch.cuda.synchronize()
        ev.append(("step", before, snap(st), (model, prm, float(out.sum().item()), y_k.cpu().numpy()[0])))
        return out

    def rep(ctx_, st, to, stream=None):
        before = snap(st)
        orig_rep(ctx_, st, to, stream=stream)
        torch.cuda.synchronize()
        ev.append(("reparam", before, snap(st), (to,)))

    def ds(ctx_, y, f, out=None, stream=None):
        o = orig_ds(ctx_, y, f, out=out, stream=stream)
        ev.append(("downsample", None, None, (f, o.cpu().numpy()[0])))
        return o

    mp.setattr(api, "step", step)
    mp.setattr(api, "softplus_reparam", rep)
    mp.setattr(api, "downsample", ds)
    res = r.run()
    mp.undo()
    return arr, init, y_real, base, ev, res


def test_driver_calls_in_schedule_order(run):
    *_, ev, res = run
    kinds = [e[0] for e in ev]
    assert kinds == (["downsample", "filter"] + ["step"] * 3 + ["grow"] + ["step"] * 3 +
                     ["downsample", "filter", "gradients", "grow"] + ["step"] * 3 + ["reparam"] +
                     ["step"] * 2 + ["reparam"])
    steps = [e[3][1] for e in ev if e[0] == "step"]
    assert [p.step for p in steps] == [1, 2, 3, 4, 5, 6, 1, 2, 3, 4, 5]
    assert [p.mask for p in steps] == [api.COARSE] * 6 + [api.ALL] * 5
    models = [e[3][0] for e in ev if e[0] == "step"]
    assert [(m.f, m.T, m.a_softplus) for m in models] == [(2, 128, 0)] * 6 + [(1, 256, 0)] * 3 + [(1, 256, 1)] * 2


def test_each_step_matches_the_oracle(run):
    arr, init, y_real, base, ev, res = run
    y_k = {}
    n_checked = dict(filter=0, grow=0, step=0, reparam=0)
    for kind, before, after, a in ev:
        if kind == "downsample":
            f, yk = a
            np.testing.assert_allclose(yk, oracle.downsample(y_real, f), rtol=1e-6,
                                       atol=1e-7 * np.abs(y_real).max())
            y_k[f] = yk
            cur_f = f
        elif kind == "filter":
            tm = osch.level(base, cur_f)
            _, keep_o, g_o = osch.filter_step(o_state(before), arr, tm, y_k[cur_f])
            keep = kept_mask(before, after)
            band = np.abs(g_o) <= 1e-6 * np.abs(g_o).max()
            assert np.array_equal(keep[~band], keep_o[~band])
            assert 0 < keep.sum() < len(keep)
            for k in api.PARAMS:
                np.testing.assert_array_equal(after["m"][k], before["m"][k][keep])
            n_checked["filter"] += 1
        elif kind == "gradients":
            tm = osch.level(base, cur_f)
            _, g = osch.loss_and_gradients(o_state(before), arr, tm, y_k[cur_f])
            for k in api.PARAMS:
                assert rel_l2(after["grad"][k], g[k]) <= 1e-4, k
        elif kind == "grow":
            dup = a[0]
            new, born, src = osch.grow_step(o_state(before), oracle.GrowthRule(dup_frac=dup, **GROWTH))
            assert len(after["balls"]["x"]) == new.count()
            for k in api.PARAMS:
                np.testing.assert_allclose(after["balls"][k], new.balls[k], rtol=0, atol=2e-6 * 6)
                np.testing.assert_array_equal(after["m"][k] == 0.0, born | (before["m"][k][src] == 0.0))
            if dup > 0:
                assert born.sum() >= 1
            n_checked["grow"] += 1
        elif kind == "step":
            model, prm, loss, yk = a
            st = o_state(before, softplus=bool(model.a_softplus))
            L, g = osch.loss_and_gradients(st, arr, otime(model), yk)
            assert loss == pytest.approx(L, rel=1e-5)
            for i, k in enumerate(api.PARAMS):
                if prm.mask & (1 << i):
                    assert rel_l2(after["grad"][k], g[k]) <= 1e-4, k
                    # Adam with the driver's step count and rate, on the GPU's gradient; the
                    # hyper-parameters are the interface's float32 values (0.999 is 0.99900001,
                    # which moves 1 - beta2 by 1.3e-5 relative)
                    f32 = lambda x: float(np.float32(x))   # noqa: E731
                    p, m, v = oracle.adam_step(before["balls"][k], after["grad"][k], before["m"][k],
                                               before["v"][k], prm.step, f32(LR[i]), f32(prm.beta1),
                                               f32(prm.beta2), f32(prm.eps))
                    np.testing.assert_allclose(after["balls"][k], p, rtol=1e-6, atol=1e-7)
                    np.testing.assert_allclose(after["m"][k], m, rtol=1e-5, atol=1e-12)
                else:
                    np.testing.assert_array_equal(after["balls"][k], before["balls"][k])
            n_checked["step"] += 1
        elif kind == "reparam":
            to = a[0]
            want = oracle.softplus_inv(before["balls"]["a"]) if to else oracle.softplus(before["balls"]["a"])
            np.testing.assert_allclose(after["balls"]["a"], want, rtol=2e-6)
            assert not after["m"]["a"].any() and not after["v"]["a"].any()
            n_checked["reparam"] += 1
    assert n_checked == dict(filter=2, grow=2, step=11, reparam=2)


def test_independent_fp64_schedule_agrees(run):
    arr, init, y_real, base, ev, res = run
    cfg = osch.Config(base=base, lr=LR, growth=dict(GROWTH), dup_frac=DUP, stages=[
        osch.Stage(f=2, mask=osch.COARSE, iters=6, filter=True, grow_every=3),
        osch.Stage(f=1, mask=osch.ALL, iters=5, filter=True, duplicate=True, softplus_frac=0.4)])
    st, recs = osch.run(init, arr, y_real, cfg)
    log = res["log"]
    gpu_losses = [[e["loss"] for e in log if e["kind"] == "iter" and e["stage"] == s] for s in (0, 1)]
    entry = [e["balls"] for e in log if e["kind"] == "stage-entry"]
    assert entry == [recs[0]["count_entry"], recs[1]["count_entry"]]
    assert res["state"].count() == st.count()
    for s in (0, 1):
        np.testing.assert_allclose(gpu_losses[s], recs[s]["losses"], rtol=1e-3)
    # the schedule did something: the loss fell in each stage
    assert all(r["losses"][-1] < r["losses"][0] for r in recs)
