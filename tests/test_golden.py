"""Stored oracle outputs (tests/golden/oracle_small.json, written by
tests/golden/make_golden.py): the oracle must keep reproducing them (a change
of its arithmetic shows here first), and the HIP path must match them to the
parity tolerances."""
import json
import os

import numpy as np
import pytest

import oracle
from _util import rel_l2

HERE = os.path.dirname(os.path.abspath(__file__))
G = json.load(open(os.path.join(HERE, "golden", "oracle_small.json")))
PROFILES = {"gauss": oracle.GAUSS, "uniform": oracle.UNIFORM}


def _inputs():
    f32 = lambda d: {k: np.asarray(v, np.float32) for k, v in d.items()}
    return f32(G["array"]), f32(G["balls"]), f32(G["gt"])


def _tm(prof):
    return oracle.Time(c=G["c"], dt=G["dt"], T=G["T"], f=1, profile=PROFILES[prof], directivity=oracle.COS,
                       K=G["K"])


@pytest.mark.parametrize("prof", ["gauss", "uniform"])
def test_oracle_reproduces_golden(prof):
    arr, balls, gt = _inputs()
    g = G[prof]
    y = oracle.simulate(balls, arr, _tm(prof))
    np.testing.assert_allclose(y, np.asarray(g["y"]), rtol=1e-12, atol=1e-15)
    gr = oracle.vjp(balls, arr, _tm(prof), np.asarray(g["v"], np.float32))
    for k, ref in g["grad"].items():
        np.testing.assert_allclose(gr[k], np.asarray(ref), rtol=1e-11, atol=1e-15)
    keep, gf, _ = oracle.filter_zero_grad(balls, arr, _tm(prof), np.asarray(g["y_ref"], np.float32))
    np.testing.assert_allclose(gf, np.asarray(g["filter_g"]), rtol=1e-11, atol=1e-15)
    np.testing.assert_array_equal(keep.astype(int), g["filter_keep"])


@pytest.mark.gpu
@pytest.mark.parametrize("prof", ["gauss", "uniform"])
def test_gpu_matches_golden(gpu, prof):
    import torch
    from paper_2601_00551_amd import api
    arr, balls, gt = _inputs()
    g = G[prof]
    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    A = {k: torch.as_tensor(v, device=dev) for k, v in arr.items()}
    B = {k: torch.as_tensor(v, device=dev) for k, v in balls.items()}
    m = api.Model(c=G["c"], dt=G["dt"], T=G["T"], f=1, profile=PROFILES[prof], directivity=api.DIR_COS,
                  gauss_K=G["K"])
    y = api.simulate_signals(ctx, A, B, m)[0].cpu().numpy()
    assert rel_l2(y, g["y"]) <= 1e-5
    v = torch.as_tensor(np.asarray(g["v"], np.float32)[None], device=dev)
    gr = api.adjoint_gradients(ctx, A, B, m, v)
    for k, ref in g["grad"].items():
        assert rel_l2(gr[k].cpu().numpy(), ref) <= 1e-4, k
    y_ref = torch.as_tensor(np.asarray(g["y_ref"], np.float32)[None], device=dev)
    out, off, gf, _ = api.filter_zero_grad(ctx, A, B, m, y_ref)
    gref = np.asarray(g["filter_g"])
    assert rel_l2(gf.cpu().numpy(), gref) <= 1e-4
    band = np.abs(gref) <= 1e-6 * np.abs(gref).max()
    keep = gf.cpu().numpy() < 0
    np.testing.assert_array_equal(keep[~band], np.asarray(g["filter_keep"], bool)[~band])
    ctx.close()
