"""Point sampling (the pressure at the sample times, GAUSS profile) and its
decimation pyramid: HIP path vs the FP64 oracle under oracle.POINT.

Same bars as the bin-average path: signals relative L2 <= 1e-5, gradients
<= 1e-4 per parameter, decimation and compaction exact.
"""
import numpy as np
import pytest
import torch

import oracle
from _util import PARAMS, gmodel, otime, rel_l2, small_scene, to_dev
from paper_2601_00551_amd import _abi, api, synth

pytestmark = pytest.mark.gpu

SIG_TOL = 1e-5
GRAD_TOL = 1e-4
PT = api.SAMPLING_POINT


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def pm(T, **kw):
    return gmodel(T, sampling=PT, **kw)


def pt(T, **kw):
    return otime(T, sampling=oracle.POINT, **kw)


def run_fwd(ctx, arr, balls, m, **kw):
    dev = torch.device("cuda:0")
    return api.simulate_signals(ctx, to_dev(arr, dev), to_dev(balls, dev), m, **kw)


def run_adj(ctx, arr, balls, m, v, mask=api.ALL, **kw):
    dev = torch.device("cuda:0")
    g = api.adjoint_gradients(ctx, to_dev(arr, dev), to_dev(balls, dev), m,
                              torch.as_tensor(v, dtype=torch.float32, device=dev).contiguous(), mask=mask, **kw)
    return {k: (None if t is None else t.cpu().numpy()) for k, t in g.items()}


@pytest.mark.parametrize("directivity", [1, 0])
def test_point_forward_matches_oracle(ctx, directivity):
    # 5000 balls (ragged last chunk), 37 transducers, record cut at T = 450
    arr, balls = small_scene(211 + directivity)
    T = 450
    y = run_fwd(ctx, arr, balls, pm(T, directivity=directivity))[0].cpu().numpy()
    ref = oracle.simulate(balls, arr, pt(T, directivity=directivity))
    assert np.count_nonzero(ref) > 1000
    assert rel_l2(y, ref) <= SIG_TOL
    assert np.max(np.abs(y - ref)) <= 1e-4 * np.max(np.abs(ref))
    # a different signal from the bin average of the same scene
    yb = oracle.simulate(balls, arr, otime(T, directivity=directivity))
    assert rel_l2(yb, ref) > 1e-3


def test_point_levels_and_record_start(ctx):
    arr, balls = small_scene(215, nb=3000, nd=20)
    for f, t0 in ((1, 5.0), (2, 3.3), (4, 0.0), (16, 1.0)):
        T = 2000 // f
        y = run_fwd(ctx, arr, balls, pm(T, f=f, t0=t0))[0].cpu().numpy()
        ref = oracle.simulate(balls, arr, pt(T, f=f, t0=t0))
        assert rel_l2(y, ref) <= SIG_TOL, (f, t0)


@pytest.mark.parametrize("directivity", [1, 0])
def test_point_adjoint_matches_oracle(ctx, directivity):
    arr, balls = small_scene(221 + directivity, nb=3000, nd=29)
    T = 450
    v = np.random.default_rng(17).normal(size=(29, T)).astype(np.float32)
    g = run_adj(ctx, arr, balls, pm(T, directivity=directivity), v)
    ref = oracle.vjp(balls, arr, pt(T, directivity=directivity), v)
    for k in PARAMS:
        assert rel_l2(g[k], ref[k]) <= GRAD_TOL, (k, rel_l2(g[k], ref[k]))


def test_point_adjoint_masks(ctx):
    arr, balls = small_scene(231, nb=1500, nd=17)
    T = 450
    v = np.random.default_rng(2).normal(size=(17, T)).astype(np.float32)
    ref = oracle.vjp(balls, arr, pt(T), v)
    for mask in (api.P0, api.XYZ, api.COARSE, api.A | api.X):
        g = run_adj(ctx, arr, balls, pm(T), v, mask=mask)
        for i, k in enumerate(PARAMS):
            if mask & (1 << i):
                assert rel_l2(g[k], ref[k]) <= GRAD_TOL, (mask, k)
            else:
                assert g[k] is None


@pytest.mark.parametrize("tuning", [
    dict(fwd_dets=1, fwd_block=64, fwd_bpt=1, adj_dets=1, adj_block=64, adj_bpt=1),
    dict(fwd_dets=3, fwd_block=256, fwd_bpt=4, fwd_grid=7, adj_dets=5, adj_block=512, adj_bpt=3, adj_grid=3),
    dict(fwd_dets=2, fwd_tile=128, adj_dets=3, adj_tile=100),
])
def test_point_launch_shapes_agree(ctx, tuning):
    arr, balls = small_scene(241, nb=2100, nd=19)
    T = 500
    old = ctx.tuning
    try:
        ctx.tuning = tuning
        y = run_fwd(ctx, arr, balls, pm(T))[0].cpu().numpy()
        v = np.random.default_rng(3).normal(size=(19, T)).astype(np.float32)
        g = run_adj(ctx, arr, balls, pm(T), v)
    finally:
        ctx.tuning = old
    assert rel_l2(y, oracle.simulate(balls, arr, pt(T))) <= SIG_TOL
    ref = oracle.vjp(balls, arr, pt(T), v)
    for k in PARAMS:
        assert rel_l2(g[k], ref[k]) <= GRAD_TOL, k


def test_point_long_record_tiled_in_time(ctx):
    arr, balls = small_scene(251, nb=400, nd=6)
    T = 20000
    m, tm = pm(T, dt=0.0015), pt(T, dt=0.0015)
    y = run_fwd(ctx, arr, balls, m)[0].cpu().numpy()
    assert rel_l2(y, oracle.simulate(balls, arr, tm)) <= SIG_TOL
    v = np.random.default_rng(T).normal(size=(6, T)).astype(np.float32)
    g = run_adj(ctx, arr, balls, m, v)
    gr = oracle.vjp(balls, arr, tm, v)
    for k in PARAMS:
        assert rel_l2(g[k], gr[k]) <= GRAD_TOL, k


def test_point_forward_bitwise_reproducible(ctx):
    arr, balls = small_scene(261, nb=5000, nd=23)
    T = 700
    ys = []
    old = ctx.tuning
    try:
        for t in (dict(fwd_dets=4, fwd_block=512, fwd_bpt=4),
                  dict(fwd_dets=1, fwd_block=256, fwd_bpt=1),
                  dict(fwd_dets=8, fwd_block=128, fwd_bpt=2, fwd_grid=7)):
            ctx.tuning = t
            ys.append(run_fwd(ctx, arr, balls, pm(T))[0].cpu().numpy())
    finally:
        ctx.tuning = old
    for y in ys[1:]:
        assert np.array_equal(y, ys[0])


def test_point_softplus_parameterisation(ctx):
    arr, balls = small_scene(321, nb=1200, nd=15)
    T = 450
    at = oracle.softplus_inv(balls["a"]).astype(np.float32)
    b2 = dict(balls, a=at)
    m = pm(T, a_softplus=1)
    ob = dict(balls, a=oracle.softplus(at))
    assert rel_l2(run_fwd(ctx, arr, b2, m)[0].cpu().numpy(), oracle.simulate(ob, arr, pt(T))) <= SIG_TOL
    v = np.random.default_rng(2).normal(size=(15, T)).astype(np.float32)
    g = run_adj(ctx, arr, b2, m, v)
    ref = oracle.vjp(ob, arr, pt(T), v)
    ref["a"] = ref["a"] * oracle.sigmoid(at)
    for k in PARAMS:
        assert rel_l2(g[k], ref[k]) <= GRAD_TOL, k


def test_point_frames_and_edge_cases(ctx):
    """Three frames (one empty); one ball seen by one transducer over a few
    samples; a transducer inside the support; a dead ball."""
    rng = np.random.default_rng(331)
    arr = synth.hemisphere_array(23, 12.0, rng, tilt_deg=20)
    parts = [synth.uniform_balls(rng, n, 4.0, 0.15) for n in (1700, 0, 2300)]
    balls = synth.concat_balls(parts)
    off = np.array([0, 1700, 1700, 4000])
    T = 450
    dev = torch.device("cuda:0")
    y = run_fwd(ctx, arr, balls, pm(T), ball_off=torch.tensor(off, device=dev)).cpu().numpy()
    v = rng.normal(size=(3, 23, T)).astype(np.float32)
    g = run_adj(ctx, arr, balls, pm(T), v, ball_off=torch.tensor(off, device=dev))
    assert y.shape == (3, 23, T) and np.all(y[1] == 0.0)
    for f in (0, 2):
        assert rel_l2(y[f], oracle.simulate(parts[f], arr, pt(T))) <= SIG_TOL
        ref = oracle.vjp(parts[f], arr, pt(T), v[f])
        for k in PARAMS:
            assert rel_l2(g[k][off[f]:off[f + 1]], ref[k]) <= GRAD_TOL
    one = {"x": np.array([0.0], np.float32), "y": np.array([0.0], np.float32), "z": np.array([0.0], np.float32),
           "p0": np.array([1.0], np.float32), "a": np.array([0.15], np.float32)}
    a1 = {k: w[:1] for k, w in arr.items()}
    rho = float(np.sqrt(a1["qx"][0] ** 2 + a1["qy"][0] ** 2 + a1["qz"][0] ** 2))
    scale = np.abs(oracle.simulate(one, a1, pt(80, t0=rho / 1.5 - 1.0))).max()
    for T1, dt0 in ((1, 0.05), (2, -0.1), (7, 0.2), (7, -0.0123)):
        t0 = rho / 1.5 + dt0
        yo = run_fwd(ctx, a1, one, pm(T1, t0=t0))[0].cpu().numpy()
        ref = oracle.simulate(one, a1, pt(T1, t0=t0))
        assert yo.shape == ref.shape and np.max(np.abs(yo - ref)) <= 1e-5 * scale, (T1, dt0)
    near = dict(one, x=np.array([a1["qx"][0] + 0.2], np.float32), y=a1["qy"].copy(), z=a1["qz"].copy())
    assert np.all(run_fwd(ctx, a1, near, pm(50))[0].cpu().numpy() == 0)
    gn = run_adj(ctx, a1, near, pm(50), np.ones((1, 50), np.float32))
    assert all(np.all(gn[k] == 0) for k in PARAMS)
    dead = dict(one, a=np.array([-0.1], np.float32))
    assert np.all(run_fwd(ctx, a1, dead, pm(50, t0=rho / 1.5 - 0.1))[0].cpu().numpy() == 0)


@pytest.mark.parametrize("directivity", [1, 0])
def test_point_f64_twins_match_oracle_tightly(ctx, directivity):
    arr, balls = small_scene(271, nb=700, nd=9)
    T = 450
    dev = torch.device("cuda:0")
    m = pm(T, directivity=directivity)
    y = api.simulate_signals_f64(ctx, to_dev(arr, dev, torch.float64), to_dev(balls, dev, torch.float64), m)
    assert rel_l2(y[0].cpu().numpy(), oracle.simulate(balls, arr, pt(T, directivity=directivity))) <= 1e-11
    v = np.random.default_rng(4).normal(size=(9, T))
    g = api.adjoint_gradients_f64(ctx, to_dev(arr, dev, torch.float64), to_dev(balls, dev, torch.float64), m,
                                  torch.as_tensor(v, device=dev).reshape(1, 9, T).contiguous())
    gr = oracle.vjp(balls, arr, pt(T, directivity=directivity), v)
    for k in PARAMS:
        assert rel_l2(g[k].cpu().numpy(), gr[k]) <= 1e-10, k


def test_point_filter_matches_oracle(ctx):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(281)
    arr = synth.hemisphere_array(31, 12.0, rng, tilt_deg=30)
    gt = synth.polyline_phantom(rng, per_line=300, half=3.5)
    init = synth.uniform_balls(rng, 4000, 4.0, 0.15, 0.0, 0.2)
    init["z"][:7] = 30.0          # behind every transducer: g == 0 exactly
    T = 450
    tm = pt(T)
    y_ref = synth.add_noise(oracle.simulate(gt, arr, tm).astype(np.float32), rng, 0.05).astype(np.float32)
    _, g_o, _ = oracle.filter_zero_grad(init, arr, tm, y_ref)
    out, off_out, g, _ = api.filter_zero_grad(ctx, to_dev(arr, dev), to_dev(init, dev), pm(T),
                                              torch.as_tensor(y_ref[None], device=dev))
    gh = g.cpu().numpy()
    assert rel_l2(gh, g_o) <= GRAD_TOL
    assert np.all(gh[:7] == 0.0)
    keep = gh < 0
    band = np.abs(g_o) <= 1e-6 * np.max(np.abs(g_o))
    assert np.array_equal(keep[~band], (g_o < 0)[~band])
    n = int(off_out[1].item())
    assert n == keep.sum() and 0 < n < 4000
    for k in PARAMS:
        assert np.array_equal(out[k][:n].cpu().numpy(), init[k][keep])


def test_point_step_equals_composed_oracle(ctx):
    dev = torch.device("cuda:0")
    arr, balls = small_scene(291, nb=1500, nd=21)
    rng = np.random.default_rng(12)
    T = 450
    gt = dict(balls, p0=(balls["p0"] * rng.uniform(0.5, 1.5, len(balls["p0"]))).astype(np.float32))
    y_ref = oracle.simulate(gt, arr, pt(T)).astype(np.float32)
    st = api.State(balls, device=dev)
    y_work = torch.empty(1, 21, T, device=dev)
    prm = api.AdamParams(lr=(0.001, 0.001, 0.001, 0.02, 0.001), step=1)
    loss = api.step(ctx, to_dev(arr, dev), st, pm(T), torch.as_tensor(y_ref[None], device=dev), y_work, prm)
    L, v = oracle.residual_loss(oracle.simulate(balls, arr, pt(T)), y_ref)
    g = oracle.vjp(balls, arr, pt(T), v)
    assert loss[0].item() == pytest.approx(L, rel=1e-5)
    for k in PARAMS:
        assert rel_l2(st.grad[k][:len(g[k])].cpu().numpy(), g[k]) <= GRAD_TOL, k


def test_decimate_is_exact(ctx):
    dev = torch.device("cuda:0")
    y = np.random.default_rng(5).normal(size=(2, 7, 1003)).astype(np.float32)
    for f in (1, 2, 3, 4, 16, 1003):
        out = api.decimate(ctx, torch.as_tensor(y, device=dev), f).cpu().numpy()
        ref = oracle.decimate(y, f)
        assert out.shape == ref.shape
        assert np.array_equal(out, ref.astype(np.float32))


def test_point_pyramid_on_gpu(ctx):
    """Decimate_f of the full-rate point-sampled record equals the point-sampled
    record at the level."""
    arr, balls = small_scene(301, nb=1000, nd=11)
    y = run_fwd(ctx, arr, balls, pm(1600))
    for f in (2, 4, 16):
        yd = api.decimate(ctx, y, f).cpu().numpy()
        yk = run_fwd(ctx, arr, balls, pm(1600 // f, f=f)).cpu().numpy()
        assert rel_l2(yd, yk) <= 2 * SIG_TOL


def test_uniform_point_is_rejected(ctx):
    arr, balls = small_scene(311, nb=50, nd=3)
    with pytest.raises(_abi.SbpError, match="GAUSS"):
        run_fwd(ctx, arr, balls, pm(100, profile=0))


def test_point_step_graph_replays_match_eager(ctx):
    """The captured iteration under point sampling: replays, with eager work
    between them, track an eager run of the same iterations."""
    dev = torch.device("cuda:0")
    arr, balls = small_scene(341, nb=2000, nd=17)
    T = 452
    gt = dict(balls, p0=(balls["p0"] * 0.7).astype(np.float32))
    y_ref = torch.as_tensor(oracle.simulate(gt, arr, pt(T)).astype(np.float32)[None], device=dev)
    prm = api.AdamParams(lr=(0.001, 0.001, 0.001, 0.01, 0.001), step=1)
    A = to_dev(arr, dev)
    st_e = api.State(balls, device=dev)
    st_g = api.State(balls, device=dev)
    yw_e = torch.empty(1, 17, T, device=dev)
    yw_g = torch.empty(1, 17, T, device=dev)
    graph = api.StepGraph(ctx, A, st_g, pm(T), y_ref, yw_g, prm, iters=3, step0=1)
    losses_e = []
    step = 1
    for rep in range(3):
        for _ in range(3):
            prm.step = step
            losses_e.append(api.step(ctx, A, st_e, pm(T), y_ref, yw_e, prm)[0].item())
            step += 1
        graph.launch()
        graph.stream.synchronize()
        _ = (yw_e * 2).sum().item()
        np.testing.assert_allclose(graph.loss.cpu().numpy(), losses_e[-3:], rtol=1e-4)
        for k in PARAMS:
            a = st_g.balls[k].cpu().numpy()
            b = st_e.balls[k].cpu().numpy()
            assert np.max(np.abs(a - b)) <= 1e-5 * max(1.0, np.abs(b).max()), (rep, k)
    assert losses_e[-1] < losses_e[0]
    graph.close()
