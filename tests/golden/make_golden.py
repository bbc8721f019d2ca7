"""Writes oracle_small.json: seeded inputs and the FP64 oracle's outputs on
them (signals of Simulate, sections 4.2/4.3; the vector-Jacobian product of
the backpropagation, Algorithm 1; the zero-gradient filter's gradient and
decisions, section 4.2).  Calls only oracle/ and the seeded generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2601_00551_amd import synth  # noqa: E402   (seeded generators only)


def main():
    rng = np.random.default_rng(20260101)
    arr = synth.hemisphere_array(8, 12.0, rng, tilt_deg=20.0)
    balls = synth.uniform_balls(rng, 40, 3.0, 0.15)
    balls["a"] = (balls["a"] * rng.uniform(0.7, 1.3, 40)).astype(np.float32)
    gt = synth.uniform_balls(rng, 30, 2.5, 0.12)
    T, dt = 300, 0.05
    out = {"note": "written by tests/golden/make_golden.py from the FP64 oracle; inputs are float32",
           "T": T, "dt": dt, "c": 1.5, "K": 5.0,
           "array": {k: [float(x) for x in v] for k, v in arr.items()},
           "balls": {k: [float(x) for x in v] for k, v in balls.items()},
           "gt": {k: [float(x) for x in v] for k, v in gt.items()}}
    for name, prof in (("gauss", oracle.GAUSS), ("uniform", oracle.UNIFORM)):
        tm = oracle.Time(c=1.5, dt=dt, T=T, f=1, profile=prof, directivity=oracle.COS, K=5.0)
        y = oracle.simulate(balls, arr, tm)
        v = np.random.default_rng(7).normal(size=(8, T)).astype(np.float32)
        g = oracle.vjp(balls, arr, tm, v)
        y_ref = oracle.simulate(gt, arr, tm).astype(np.float32)
        keep, gf, _ = oracle.filter_zero_grad(balls, arr, tm, y_ref)
        out[name] = {"y": y.tolist(), "v": v.astype(np.float64).tolist(),
                     "grad": {k: g[k].tolist() for k in g}, "y_ref": y_ref.astype(np.float64).tolist(),
                     "filter_g": gf.tolist(), "filter_keep": keep.astype(int).tolist()}
    with open(os.path.join(HERE, "oracle_small.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
