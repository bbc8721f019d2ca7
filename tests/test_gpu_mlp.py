"""GPU parity of the growth-proposal network and its feature kernels against
the CPU reference (oracle/mlp.py, oracle/proposal.py), through the C-ABI.

Tolerances.  Both sides round inputs, weights and hidden activations to BF16,
and in the backward the back-propagated gradients fed to the matrix cores
(dL/dh per hidden layer, the output gradient in the last weight gradient);
the GPU accumulates in FP32 in the matrix cores' order, so a value that lies
within FP32 rounding of a BF16 rounding boundary can land one BF16 ulp (2^-8
relative) apart.  That is rare, hence outputs and gradients within 1e-3
relative L2 (per parameter block)."""
import numpy as np
import pytest
import torch

from oracle import adam_step
from oracle import mlp as om
from oracle import proposal as op
from paper_2601_00551_amd import api, proposal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _params(seed):
    rng = np.random.default_rng(seed)
    P = {}
    for name, shape in om.SHAPES:
        fan = 31 if name == "W1" else shape[0]
        P[name] = rng.normal(0, np.sqrt(2.0 / fan), size=shape) if name.startswith("W") \
            else rng.normal(0, 0.1, size=shape)
    P["W1"][31, :] = 0.0
    return om.pack(P).astype(np.float32)


def _blocks(g):
    u = om.unpack(g)
    return {k: u[k] for k, _ in om.SHAPES}


@pytest.mark.parametrize("M", [1, 63, 64, 65, 1000, 4097])
def test_forward_matches_oracle(ctx, M):
    dev = torch.device("cuda:0")
    p = _params(M)
    X = np.random.default_rng(100 + M).normal(size=(M, 31)).astype(np.float32)
    net = proposal.ProposalMLP(ctx, params=p)
    out = net.forward(torch.as_tensor(X, device=dev)).cpu().numpy()
    ref, _ = om.forward(p, X)
    assert rel_l2(out, ref) <= 1e-3, (M, rel_l2(out, ref))


def test_forward_exact_abs_network(ctx):
    """The |x| network of the reference pins: exact on integer inputs."""
    P = {name: np.zeros(shape) for name, shape in om.SHAPES}
    for i in range(31):
        P["W1"][i, i] = 1.0
        P["W1"][i, 31 + i] = -1.0
    P["W2"][np.arange(62), np.arange(62)] = 1.0
    P["W3"][np.arange(62), np.arange(62)] = 1.0
    P["W4"][:62, 0] = 1.0
    P["W4"][:31, 1] = 1.0
    P["b4"][:] = [0.5, -2.0]
    X = np.random.default_rng(1).integers(-8, 9, size=(130, 31)).astype(np.float32)
    net = proposal.ProposalMLP(ctx, params=om.pack(P).astype(np.float32))
    out = net.forward(torch.as_tensor(X, device="cuda:0")).cpu().numpy()
    np.testing.assert_array_equal(out[:, 0], np.abs(X).sum(1) + 0.5)
    np.testing.assert_array_equal(out[:, 1], np.maximum(X, 0).sum(1) - 2.0)


@pytest.mark.parametrize("M", [64, 777, 5000, 70000])   # 1, 1, 5 and 69 slices of rows
def test_loss_and_backward_match_oracle(ctx, M):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(200 + M)
    p = _params(300 + M)
    X = rng.normal(size=(M, 31)).astype(np.float32)
    yg = (rng.uniform(size=M) > 0.7).astype(np.float32)
    yp = rng.uniform(0, 1, size=M).astype(np.float32)
    net = proposal.ProposalMLP(ctx, params=p)
    loss, out = net.loss_and_grad(torch.as_tensor(X, device=dev), torch.as_tensor(yg, device=dev),
                                  torch.as_tensor(yp, device=dev), pos_weight=2.5)
    g = net.grad.cpu().numpy()
    ref_out, cache = om.forward(p, X)
    # the loss and its output gradient are evaluated at the GPU's outputs
    L, d = om.loss(out.cpu().numpy().astype(np.float64), yg, yp, 2.5)
    assert float(loss.item()) == pytest.approx(L, rel=1e-5)
    gref = om.backward(cache, d)
    got, ref = _blocks(g), _blocks(gref)
    for k in ref:
        assert rel_l2(got[k], ref[k]) <= 1e-3, (k, rel_l2(got[k], ref[k]))


def test_adam_matches_oracle(ctx):
    dev = torch.device("cuda:0")
    p = _params(9)
    net = proposal.ProposalMLP(ctx, params=p)
    rng = np.random.default_rng(10)
    m = np.zeros(om.NPARAM)
    v = np.zeros(om.NPARAM)
    ref = p.astype(np.float64)
    for step in (1, 2, 3):
        g = rng.normal(size=om.NPARAM).astype(np.float32)
        net.grad.copy_(torch.as_tensor(g, device=dev))
        net.adam(lr=1e-3)
        ref, m, v = adam_step(ref, g, m, v, step, 1e-3)
        got = net.params.cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-7)
    # the BF16 working copy follows the parameters: forward equals a fresh network's
    X = torch.as_tensor(rng.normal(size=(100, 31)).astype(np.float32), device=dev)
    fresh = proposal.ProposalMLP(ctx, params=net.params.cpu().numpy())
    torch.testing.assert_close(net.forward(X), fresh.forward(X), rtol=0, atol=0)


def test_training_learns_a_rule(ctx):
    """A learnable labelling (grow iff feature 0 > 0.3, target p0 = 1 + feature 1)
    is fitted by the GPU training loop."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    n = 32768
    X = rng.normal(size=(n, 31)).astype(np.float32)
    yg = (X[:, 0] > 0.3).astype(np.float32)
    yp = (1.0 + X[:, 1]).astype(np.float32) * yg
    net = proposal.ProposalMLP(ctx, seed=3)
    hist = proposal.train(net, X, yg, yp, epochs=8, batch=4096, lr=2e-3, log=lambda *a, **k: None)
    assert hist[-1] < 0.2 * hist[0], hist
    Xt = rng.normal(size=(4000, 31)).astype(np.float32)
    out = net.forward(torch.as_tensor(Xt, device=dev)).cpu().numpy()
    acc = np.mean((out[:, 0] > 0) == (Xt[:, 0] > 0.3))
    assert acc > 0.95, acc


# ---------------------------------------------------- features & sites --

def _cloud(rng, g, n):
    half = g.h * g.nx / 2
    b = {k: rng.uniform(-half * 0.6, half * 0.6, n).astype(np.float32) for k in ("x", "y", "z")}
    b["p0"] = rng.uniform(0.0, 1.0, n).astype(np.float32)
    b["a"] = np.full(n, 0.1, np.float32)
    return b


def test_grid_candidates_features_append(ctx):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(12)
    g = proposal.Grid.cube(2.0, 0.2)          # 20^3 cells
    og = op.Grid(g.ox, g.oy, g.oz, g.h, g.nx, g.ny, g.nz)
    b = _cloud(rng, g, 300)
    st = api.State(b, capacity=4000, device=dev)
    mass = proposal.grid_mass(ctx, st.balls, st.ball_off, g, B_cap=st.B_cap)
    m_gpu = mass.cpu().numpy().reshape(g.nx, g.ny, g.nz)
    np.testing.assert_allclose(m_gpu, op.grid_mass(og, b), rtol=1e-6, atol=1e-6)
    # candidate decisions are taken on the GPU's own masses on both sides
    sites, M = proposal.candidates(ctx, g, mass, 0.1, a_probe=0.1)
    flat, centre = op.candidates(og, m_gpu.astype(np.float64), 0.1)
    assert M == len(flat) > 0
    xyz = torch.stack([sites[k][:M] for k in ("x", "y", "z")], 1).cpu().numpy()
    np.testing.assert_allclose(xyz, centre, rtol=0, atol=1e-6)
    np.testing.assert_array_equal(sites["p0"][:M].cpu().numpy(), 1.0)
    np.testing.assert_array_equal(sites["a"][:M].cpu().numpy(), np.float32(0.1))
    # features from given probe gradients
    gr = {k: torch.as_tensor(rng.normal(size=M).astype(np.float32), device=dev) for k in api.PARAMS}
    X = proposal.features(ctx, g, mass, sites, M, gr, half=2.0).cpu().numpy()
    Xr = op.features(og, m_gpu.astype(np.float64), xyz.astype(np.float64), gr["p0"].cpu().numpy(),
                     torch.stack([gr["x"], gr["y"], gr["z"]], 1).cpu().numpy(), 2.0)
    np.testing.assert_allclose(X, Xr, rtol=2e-6, atol=2e-7)
    # append: decisions on the GPU's logits; order and values as the reference
    out = torch.as_tensor(rng.normal(size=(M, 2)).astype(np.float32), device=dev)
    n_new = proposal.append_proposals(ctx, st, sites, out, M, a_init=0.1, p0_scale=0.75)
    ref = op.append(b, xyz.astype(np.float64), out.cpu().numpy(), 0.1, p0_scale=0.75)
    assert n_new == len(ref["x"]) == st.count()
    for k in api.PARAMS:
        np.testing.assert_allclose(st.balls[k][:n_new].cpu().numpy(), ref[k], rtol=1e-7, atol=1e-7)
        assert float(st.m[k][300:n_new].abs().max()) == 0.0
    # the capacity error leaves the state unchanged
    small = api.State(b, capacity=301, device=dev)
    with pytest.raises(Exception):
        proposal.append_proposals(ctx, small, sites, out, M, a_init=0.1)
    assert small.count() == 300


def test_candidates_capacity_and_empty(ctx):
    dev = torch.device("cuda:0")
    g = proposal.Grid.cube(1.0, 0.25)
    mass = torch.zeros(g.ncell, device=dev)
    _, M = proposal.candidates(ctx, g, mass, 0.1, a_probe=0.1)
    assert M == 0
    mass[(3 * 8 + 3) * 8 + 3] = 1.0
    sites = {k: torch.empty(10, device=dev) for k in api.PARAMS}
    with pytest.raises(Exception):
        proposal.candidates(ctx, g, mass, 0.1, a_probe=0.1, sites=sites)
    _, M = proposal.candidates(ctx, g, mass, 0.1, a_probe=0.1)
    assert M == 26


def test_probe_features_follow_oracle_gradients(ctx):
    """End to end on a small measurement: the probe back-projection feature
    equals the oracle's -dL/dp0 of unit balls at the sites, normalised."""
    import oracle
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(13)
    from paper_2601_00551_amd import synth
    arr = synth.hemisphere_array(16, 12.0, rng)
    g = proposal.Grid.cube(1.0, 0.25)
    b = _cloud(rng, g, 40)
    b["a"][:] = 0.2
    model = api.Model(c=1.5, dt=0.05, T=300, f=1)
    A = {k: torch.as_tensor(v, device=dev) for k, v in arr.items()}
    st = api.State(b, capacity=100, device=dev)
    yref = torch.as_tensor(rng.normal(size=(1, 16, 300)).astype(np.float32) * 0.01, device=dev)
    yw = torch.empty(1, 16, 300, device=dev)
    api.simulate_signals(ctx, A, st.balls, model, ball_off=st.ball_off, y=yw, B_cap=st.B_cap)
    api.residual_loss(ctx, yw, yref, v_out=yw)
    fb = proposal.FeatureBuilder(ctx, g, occ=0.1, a_probe=0.2, half=1.0)
    M, X, sites = fb.build(A, st, model, yw)
    assert M > 0
    v = yw.cpu().numpy()[0].astype(np.float64)
    probe = {k: sites[k][:M].cpu().numpy().astype(np.float64) for k in api.PARAMS}
    tm = oracle.Time(c=1.5, dt=0.05, T=300, f=1)
    gref = oracle.vjp(probe, {k: np.asarray(x, np.float64) for k, x in arr.items()}, tm, v)
    f0 = -gref["p0"] / np.max(np.abs(gref["p0"]))
    assert rel_l2(X[:, 0].cpu().numpy(), f0) <= 1e-4
    gn = np.sqrt(gref["x"] ** 2 + gref["y"] ** 2 + gref["z"] ** 2)
    assert rel_l2(X[:, 1].cpu().numpy(), gn / gn.max()) <= 1e-4
