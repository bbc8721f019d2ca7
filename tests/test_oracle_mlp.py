"""Pins of the CPU reference of the growth-proposal network and of its
candidate-site / feature definitions (no GPU).

The network is not in the paper, so nothing the paper prints pins it; these
tests pin the reference to library routines (torch's bfloat16 conversion and
autograd), closed forms (networks built to compute a known function, the loss
at z = 0), finite differences and hand-countable grid cases."""
import numpy as np
import pytest
import torch

from oracle import mlp as om
from oracle import proposal as op


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, -1e-42]]).astype(np.float32)
    # exact ties: a float32 whose low 16 bits are 0x8000
    ties = (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = om.bf16_round(x)
    np.testing.assert_array_equal(got, ref)


def test_layout_size():
    assert om.NPARAM == 140546
    p = np.arange(om.NPARAM, dtype=np.float64)
    np.testing.assert_array_equal(om.pack(om.unpack(p)), p)
    u = om.unpack(p)
    assert u["b1"][0] == 8192 and u["W2"][0, 0] == 8448 and u["b4"][1] == 140545


def _zero_params():
    return {name: np.zeros(shape) for name, shape in om.SHAPES}


def test_abs_sum_network():
    """W1 = [I, -I] and ReLU give |x_i|; W2 = W3 = I pass it on; W4 sums: out0 =
    sum |x_i| exactly for bf16-representable inputs (small integers)."""
    P = _zero_params()
    for i in range(31):
        P["W1"][i, i] = 1.0
        P["W1"][i, 31 + i] = -1.0
    P["W2"][np.arange(62), np.arange(62)] = 1.0
    P["W3"][np.arange(62), np.arange(62)] = 1.0
    P["W4"][:62, 0] = 1.0
    P["W4"][:31, 1] = 1.0
    P["b4"][:] = [0.5, -2.0]
    rng = np.random.default_rng(1)
    X = rng.integers(-8, 9, size=(50, 31)).astype(np.float64)
    out, _ = om.forward(om.pack(P), X)
    np.testing.assert_array_equal(out[:, 0], np.abs(X).sum(1) + 0.5)
    np.testing.assert_array_equal(out[:, 1], np.maximum(X, 0).sum(1) - 2.0)


def test_zero_weights_give_bias():
    P = _zero_params()
    P["b4"][:] = [1.25, -0.75]
    P["b1"][:] = 3.0
    out, _ = om.forward(om.pack(P), np.random.default_rng(2).normal(size=(7, 31)))
    np.testing.assert_array_equal(out, np.tile([1.25, -0.75], (7, 1)))


def test_loss_closed_form():
    out = np.array([[0.0, 0.3], [0.0, 2.0], [50.0, 0.0]])
    yg = np.array([1.0, 0.0, 0.0])
    yp = np.array([0.5, 9.0, 0.0])
    L, d = om.loss(out, yg, yp, pos_weight=3.0)
    ref = (3.0 * np.log(2) + 0.04 + np.log(2) + (50.0 + np.log1p(np.exp(-50.0)))) / 3
    assert L == pytest.approx(ref, rel=1e-14)
    # d/dz at z = 0: pos_weight * (1/2 - 1) for y = 1, 1/2 for y = 0; d/dp = 2 (p - t) y
    np.testing.assert_allclose(d[:, 0], np.array([-1.5, 0.5, 1.0]) / 3, rtol=1e-12)
    np.testing.assert_allclose(d[:, 1], np.array([2 * (0.3 - 0.5), 0.0, 0.0]) / 3, rtol=1e-12)


def test_loss_gradient_finite_difference():
    rng = np.random.default_rng(3)
    out = rng.normal(size=(20, 2))
    yg = (rng.uniform(size=20) > 0.5).astype(float)
    yp = rng.uniform(size=20)
    _, d = om.loss(out, yg, yp, 2.5)
    eps = 1e-6
    for idx in [(0, 0), (3, 1), (7, 0), (19, 1)]:
        o1, o2 = out.copy(), out.copy()
        o1[idx] += eps
        o2[idx] -= eps
        fd = (om.loss(o1, yg, yp, 2.5)[0] - om.loss(o2, yg, yp, 2.5)[0]) / (2 * eps)
        assert d[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def _random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = {}
    for name, shape in om.SHAPES:
        fan = 31 if name == "W1" else shape[0]
        P[name] = rng.normal(0, scale * np.sqrt(2.0 / fan), size=shape) if name.startswith("W") \
            else rng.normal(0, 0.1, size=shape)
    P["W1"][31, :] = 0.0
    return om.pack(P)


def test_backward_finite_difference_without_rounding(monkeypatch):
    """With the BF16 rounding switched off the network is smooth almost
    everywhere: central differences pin every weight block of the backward."""
    monkeypatch.setattr(om, "bf16_round", lambda x: np.asarray(x, np.float64))
    rng = np.random.default_rng(4)
    p = _random_params(5)
    X = rng.normal(size=(9, 31))
    yg = (rng.uniform(size=9) > 0.4).astype(float)
    yp = rng.uniform(size=9)

    def total(pp):
        out, _ = om.forward(pp, X)
        return om.loss(out, yg, yp, 1.7)[0]

    out, cache = om.forward(p, X)
    _, d = om.loss(out, yg, yp, 1.7)
    g = om.backward(cache, d)
    offs = {}
    o = 0
    for name, shape in om.SHAPES:
        offs[name] = o
        o += int(np.prod(shape))
    picks = [offs["W1"] + 3 * 256 + 17, offs["b1"] + 5, offs["W2"] + 1000, offs["b2"] + 200,
             offs["W3"] + 40000, offs["b3"] + 77, offs["W4"] + 2 * 100 + 1, offs["W4"] + 2 * 7, offs["b4"],
             offs["b4"] + 1]
    eps = 1e-6
    for k in picks:
        p1, p2 = p.copy(), p.copy()
        p1[k] += eps
        p2[k] -= eps
        fd = (total(p1) - total(p2)) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_backward_matches_torch_autograd_with_rounding():
    """Straight-through gradients of the rounded network, against autograd on
    a torch FP64 network whose roundings are detached offsets."""
    rng = np.random.default_rng(6)
    p = _random_params(7)
    X = rng.normal(size=(33, 31))
    yg = (rng.uniform(size=33) > 0.5).astype(float)
    yp = rng.uniform(size=33)
    out, cache = om.forward(p, X)
    L, d = om.loss(out, yg, yp, 2.0)
    g = om.backward(cache, d, round_grads=False)

    def st(t):  # value rounded to bf16, gradient passed straight through
        r = t.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
        return t + (r - t).detach()

    P = {k: torch.tensor(v, requires_grad=True) for k, v in om.unpack(p).items()}
    x = torch.zeros(33, 32, dtype=torch.float64)
    x[:, :31] = st(torch.tensor(X))
    h = x
    for i in (1, 2, 3):
        h = st(torch.relu(h @ st(P[f"W{i}"]) + P[f"b{i}"]))
    o = h @ st(P["W4"]) + P["b4"]
    np.testing.assert_allclose(o.detach().numpy(), out, rtol=1e-12, atol=1e-12)
    z, pp = o[:, 0], o[:, 1]
    y, t = torch.tensor(yg), torch.tensor(yp)
    Lt = torch.mean(2.0 * y * torch.nn.functional.softplus(-z) + (1 - y) * torch.nn.functional.softplus(z)
                    + y * (pp - t) ** 2)
    Lt.backward()
    assert float(Lt) == pytest.approx(L, rel=1e-12)
    ref = np.concatenate([P[name].grad.numpy().ravel() for name, _ in om.SHAPES])
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-13)


def test_backward_gradient_rounding_matches_torch_bfloat16_hooks():
    """The rounded back-propagation against autograd on the same torch FP64
    network, with torch's own bfloat16 conversion applied by gradient hooks to
    dL/dh3, dL/dh2 and dL/dh1 (the operands of the next products) and to the
    output gradient in the last layer's weight gradient."""
    rng = np.random.default_rng(16)
    p = _random_params(17)
    X = rng.normal(size=(41, 31))
    yg = (rng.uniform(size=41) > 0.5).astype(float)
    yp = rng.uniform(size=41)
    out, cache = om.forward(p, X)
    _, d = om.loss(out, yg, yp, 1.5)
    g = om.unpack(om.backward(cache, d))

    def tbf(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    def st(t):
        return t + (tbf(t.detach()) - t).detach()

    P = {k: torch.tensor(v, requires_grad=True) for k, v in om.unpack(p).items()}
    x = torch.zeros(41, 32, dtype=torch.float64)
    x[:, :31] = st(torch.tensor(X))
    hs, h = [], x
    for i in (1, 2, 3):
        h = st(torch.relu(h @ st(P[f"W{i}"]) + P[f"b{i}"]))
        h.register_hook(tbf)
        hs.append(h)
    o = h @ st(P["W4"]) + P["b4"]
    o.backward(torch.tensor(d))
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "b4"):
        np.testing.assert_allclose(g[name], P[name].grad.numpy(), rtol=1e-10, atol=1e-14, err_msg=name)
    gw4 = hs[2].detach().T @ tbf(torch.tensor(d))
    np.testing.assert_allclose(g["W4"], gw4.numpy(), rtol=1e-10, atol=1e-14)
    # and the rounding is not vacuous here: the straight-through gradients differ
    g0 = om.unpack(om.backward(cache, d, round_grads=False))
    assert not np.allclose(g0["W1"], g["W1"], rtol=1e-6, atol=0)


def test_backward_rounding_is_exact_on_bf16_representable_gradients():
    """Small-integer weights and inputs with an output gradient of powers of two
    keep every back-propagated value exactly representable in BF16: the
    rounded and the plain back-propagation agree with autograd exactly."""
    rng = np.random.default_rng(18)
    P = {name: rng.integers(-1, 2, size=shape).astype(np.float64) for name, shape in om.SHAPES}
    for k, dens in (("W1", 0.2), ("W2", 0.02), ("W3", 0.02)):
        P[k] *= rng.uniform(size=P[k].shape) < dens       # sparse: activations stay below 256
    p = om.pack(P)
    X = rng.integers(-1, 2, size=(12, 31)).astype(np.float64)
    out, cache = om.forward(p, X)
    assert max(np.abs(h).max() for h in cache[1:4]) < 256 and np.abs(cache[3]).max() > 0
    d = 2.0 ** rng.integers(-6, -2, size=(12, 2)) * rng.choice([-1.0, 1.0], size=(12, 2))
    g = om.backward(cache, d)
    np.testing.assert_array_equal(g, om.backward(cache, d, round_grads=False))
    Pt = {k: torch.tensor(v, requires_grad=True) for k, v in P.items()}
    x = torch.zeros(12, 32, dtype=torch.float64)
    x[:, :31] = torch.tensor(X)
    h = x
    for i in (1, 2, 3):
        h = torch.relu(h @ Pt[f"W{i}"] + Pt[f"b{i}"])
    (h @ Pt["W4"] + Pt["b4"]).backward(torch.tensor(d))
    ref = np.concatenate([Pt[name].grad.numpy().ravel() for name, _ in om.SHAPES])
    np.testing.assert_array_equal(g, ref)


# ----------------------------------------------------------- grid cases --

def _grid(n=6, h=0.5):
    return op.Grid(-n * h / 2, -n * h / 2, -n * h / 2, h, n, n, n)


def _ball_at_cell(g, i, j, k, p0=1.0):
    return {"x": np.array([g.ox + (i + 0.5) * g.h]), "y": np.array([g.oy + (j + 0.5) * g.h]),
            "z": np.array([g.oz + (k + 0.5) * g.h]), "p0": np.array([p0]), "a": np.array([0.1])}


def test_single_occupied_cell_has_26_candidates():
    g = _grid()
    m = op.grid_mass(g, _ball_at_cell(g, 2, 3, 2, 0.7))
    assert m.sum() == pytest.approx(0.7) and m[2, 3, 2] == pytest.approx(0.7)
    flat, centre = op.candidates(g, m, 0.1)
    assert len(flat) == 26
    assert np.all(np.diff(flat) > 0)
    ijk = np.stack(np.unravel_index(flat, (6, 6, 6)), 1)
    assert np.all(np.abs(ijk - [2, 3, 2]).max(1) == 1)
    np.testing.assert_allclose(centre[:, 0], g.ox + (ijk[:, 0] + 0.5) * g.h)


def test_corner_cell_has_7_candidates_and_threshold():
    g = _grid()
    m = op.grid_mass(g, _ball_at_cell(g, 0, 0, 5, 0.3))
    assert len(op.candidates(g, m, 0.1)[0]) == 7
    assert len(op.candidates(g, m, 0.3)[0]) == 7      # mass >= occ is occupied
    assert len(op.candidates(g, m, 0.31)[0]) == 0


def test_mass_conserved_inside_grid():
    g = _grid(8, 0.25)
    rng = np.random.default_rng(8)
    b = {k: rng.uniform(-1.2, 1.2, 500) for k in ("x", "y", "z")}
    b["p0"] = rng.uniform(0.1, 1.0, 500)
    b["a"] = np.full(500, 0.1)
    inside = np.all(np.abs(np.stack([b["x"], b["y"], b["z"]])) < 1.0, axis=0)
    assert op.grid_mass(g, b).sum() == pytest.approx(b["p0"][inside].sum(), rel=1e-12)


def test_feature_neighbour_order_and_scales():
    g = _grid(5, 1.0)
    mass = np.zeros((5, 5, 5))
    # give each neighbour of cell (2, 2, 2) the mass 1 + its (di, dj, dk) code
    for q, (di, dj, dk) in enumerate(op.NEIGHBOURS):
        mass[2 + di, 2 + dj, 2 + dk] = 1.0 + q
    xyz = np.array([[0.0, 0.0, 0.0], [-2.2, -2.2, -2.2]])   # cells (2,2,2) and (0,0,0)
    gp = np.array([-4.0, 2.0])
    gr = np.array([[3.0, 0.0, 4.0], [0.0, 1.0, 0.0]])
    X = op.features(g, mass, xyz, gp, gr, half=2.5)
    np.testing.assert_allclose(X[:, 0], [1.0, -0.5])
    np.testing.assert_allclose(X[:, 1], [1.0, 0.2])
    np.testing.assert_allclose(X[0, 2:28], (1.0 + np.arange(26)) / 26.0)
    # corner cell (0,0,0): of its seven in-grid neighbours only (1,1,1) (code 25,
    # the last) carries mass, 1 + code of (-1,-1,-1) seen from (2,2,2) = 1
    assert X[1, 2 + 25] == pytest.approx(1.0 / 26.0)
    assert np.count_nonzero(X[1, 2:28]) == 1
    np.testing.assert_allclose(X[:, 28:], xyz / 2.5)


def test_append_order_and_values():
    sites = np.array([[0.0, 1, 2], [3, 4, 5], [6, 7, 8]])
    out = np.array([[1.0, 0.4], [-1.0, 2.0], [0.5, -0.3]])
    b = {"x": [9.0], "y": [9.0], "z": [9.0], "p0": [1.0], "a": [0.2]}
    nb = op.append(b, sites, out, 0.1)
    np.testing.assert_array_equal(nb["x"], [9.0, 0.0, 6.0])
    np.testing.assert_array_equal(nb["p0"], [1.0, 0.4, 0.0])
    np.testing.assert_array_equal(nb["a"], [0.2, 0.1, 0.1])
