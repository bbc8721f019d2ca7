"""Shared test helpers: seeded inputs as numpy (for the oracle) and torch (for
the HIP path), built from the same float32 arrays."""
import numpy as np

import oracle
from paper_2601_00551_amd import synth

PARAMS = ("x", "y", "z", "p0", "a")
AKEYS = ("qx", "qy", "qz", "nx", "ny", "nz")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def to_dev(d, device, dtype=None):
    import torch
    dt = dtype or torch.float32
    return {k: torch.as_tensor(np.ascontiguousarray(v), dtype=dt, device=device) for k, v in d.items()}


def otime(T, dt=0.025, f=1, profile=oracle.GAUSS, directivity=oracle.COS, K=5.0, t0=0.0, c=1.5,
          sampling=oracle.BIN):
    return oracle.Time(c=c, dt=dt, t0=t0, T=T, f=f, profile=profile, directivity=directivity, K=K,
                       sampling=sampling)


def gmodel(T, dt=0.025, f=1, profile=1, directivity=1, K=5.0, t0=0.0, c=1.5, a_softplus=0, sampling=0):
    from paper_2601_00551_amd.api import Model
    return Model(c=c, dt=dt, t0=t0, T=T, f=f, profile=profile, directivity=directivity, gauss_K=K,
                 a_softplus=a_softplus, sampling=sampling)


def small_scene(seed, nb=5000, nd=37, radius=12.0, half=4.0, a=0.15, tilt=25.0):
    """A few thousand balls in a cube seen by a few dozen transducers on a cap,
    with some normals tilted so that COS directivity cuts some pairs."""
    rng = np.random.default_rng(seed)
    arr = synth.hemisphere_array(nd, radius, rng, tilt_deg=tilt)
    balls = synth.uniform_balls(rng, nb, half, a)
    balls["a"] = (balls["a"] * rng.uniform(0.7, 1.3, nb)).astype(np.float32)
    return arr, balls
