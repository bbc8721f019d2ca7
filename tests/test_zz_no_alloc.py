"""The allocation-free forward, sbp_simulate_signals_noalloc, through the
C-ABI, against the allocating sbp_simulate_signals on the same inputs: the
two run the same kernels on different workspaces, so the signals must agree
bit for bit.  Two calls in a row (the second on a smaller cloud, record and
array, so that the fixed workspace holds the first call's leftovers), frames,
accumulation, and the profiles with their own accumulation forms."""
import numpy as np
import pytest
import torch

from _util import gmodel, small_scene, to_dev
from paper_2601_00551_amd import api

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = api.Context(0)
    yield c
    c.close()


def _both(ctx, arr, balls, model, **kw):
    dev = torch.device("cuda:0")
    A, B = to_dev(arr, dev), to_dev(balls, dev)
    kw1 = dict(kw)
    if "y" in kw:
        kw1["y"] = kw["y"].clone()        # the same starting values for both calls
    y0 = api.simulate_signals(ctx, A, B, model, **kw)
    y1 = api.simulate_signals(ctx, A, B, model, noalloc=True, **kw1)
    torch.cuda.synchronize()
    return y0, y1


@pytest.mark.parametrize("profile,sampling", [(1, 0), (0, 0), (1, 1)])
def test_noalloc_equals_allocating_forward_twice(ctx, profile, sampling):
    # first call: 20k balls, 40 transducers, 1500 samples; second: smaller
    for seed, nb, nd, T in ((11, 20000, 40, 1500), (12, 3000, 17, 700)):
        arr, balls = small_scene(seed, nb=nb, nd=nd)
        y0, y1 = _both(ctx, arr, balls, gmodel(T, profile=profile, sampling=sampling))
        assert torch.count_nonzero(y0).item() > 0
        assert torch.equal(y0, y1), (seed, profile, sampling)


def test_noalloc_frames_and_accumulate(ctx):
    dev = torch.device("cuda:0")
    arr, balls = small_scene(21, nb=9000, nd=23)
    off = torch.tensor([0, 4000, 4000, 9000], dtype=torch.int64, device=dev)   # one empty frame
    T = 900
    base = torch.randn(3, 23, T, device=dev)
    y0, y1 = _both(ctx, arr, balls, gmodel(T), ball_off=off, y=base.clone(), accumulate=True)
    assert torch.equal(y0, y1)
    assert torch.equal(y0[1], base[1])        # the empty frame only keeps what it held
