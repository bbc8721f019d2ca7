"""Pins of the oracle's multi-frame merge of accepted proposals
(oracle/proposal.py): hand-counted layouts, and the single-frame case equal
to the plain append."""
import numpy as np

from oracle import proposal as op


def _balls(xs):
    xs = np.asarray(xs, np.float64)
    return {"x": xs, "y": xs + 100, "z": xs + 200, "p0": xs + 300, "a": xs + 400}


def test_hand_counted_three_frames():
    # frames of 2, 0 and 3 balls; 2, 3 and 1 sites; frame 2's scale is zero
    balls = _balls([1, 2, 3, 4, 5])
    off = [0, 2, 2, 5]
    sites = np.array([[10, 11, 12], [20, 21, 22],                 # frame 0
                      [30, 31, 32], [40, 41, 42], [50, 51, 52],   # frame 1
                      [60, 61, 62]], np.float64)                  # frame 2
    out = np.array([[1.0, 0.5], [-1.0, 9.0],
                    [2.0, -3.0], [0.5, 2.0], [-0.1, 1.0],
                    [3.0, 1.0]])
    scale = [1.0, 2.0, 0.0]
    grad = np.arange(5, dtype=np.float64) + 1.0
    nb, noff, ex = op.merge(balls, off, sites, [0, 2, 5, 6], out, scale, a_init=0.25, extra={"g": grad})
    # frame 0: balls 1, 2 then site 10 (p0 0.5); frame 1: sites 30 (p0 max(-3, 0) * 2 = 0) and 40 (p0 4);
    # frame 2: balls 3, 4, 5 only
    assert noff.tolist() == [0, 3, 5, 8]
    assert nb["x"].tolist() == [1, 2, 10, 30, 40, 3, 4, 5]
    assert nb["y"].tolist() == [101, 102, 11, 31, 41, 103, 104, 105]
    assert nb["p0"].tolist() == [301, 302, 0.5, 0.0, 4.0, 303, 304, 305]
    assert nb["a"].tolist() == [401, 402, 0.25, 0.25, 0.25, 403, 404, 405]
    assert ex["g"].tolist() == [1, 2, 0, 0, 0, 3, 4, 5]


def test_empty_input_gives_the_proposals_alone():
    sites = np.array([[1, 1, 1], [2, 2, 2], [3, 3, 3]], np.float64)
    out = np.array([[1.0, 1.0], [1.0, 2.0], [-1.0, 3.0]])
    nb, noff, _ = op.merge(_balls([]), [0, 0, 0], sites, [0, 1, 3], out, [1.0, 1.0], a_init=0.1)
    assert noff.tolist() == [0, 1, 2]
    assert nb["x"].tolist() == [1, 2]


def test_single_frame_equals_append():
    rng = np.random.default_rng(3)
    balls = {k: rng.normal(size=7) for k in ("x", "y", "z", "p0", "a")}
    sites = rng.normal(size=(11, 3))
    out = rng.normal(size=(11, 2))
    nb, noff, _ = op.merge(balls, [0, 7], sites, [0, 11], out, [1.5], a_init=0.2)
    ref = op.append(balls, sites, out, 0.2, p0_scale=1.5)
    for k in ref:
        np.testing.assert_array_equal(nb[k], ref[k])
    assert noff.tolist() == [0, len(ref["x"])]
