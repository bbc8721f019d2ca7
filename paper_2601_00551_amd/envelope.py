"""Envelope mesh of an arbitrary array and the random initial cloud inside it
(the first two steps of Algorithm 1 of SlingBAG Pro).

The paper builds "a closed, polygonal envelope mesh" from the array
coordinates without saying how; the reading here is the convex hull of the
transducer positions (Qhull via scipy, once per array, on the host).  Points
are drawn uniformly in the hull's bounding box from a seeded generator and
kept when sbp_mesh_inside (ray casting on the GPU, include/sbp_image.h) finds
them inside the mesh and at least `margin` from it, until N are kept.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._abi import check, lib
from .api import _exactly, _need, _p, _stream


def envelope_mesh(array) -> np.ndarray:
    """Triangles [F, 9] (float32) of the convex hull of the transducer positions."""
    from scipy.spatial import ConvexHull
    q = np.stack([array["qx"], array["qy"], array["qz"]], axis=1).astype(np.float64)
    hull = ConvexHull(q)
    return q[hull.simplices].reshape(-1, 9).astype(np.float32)


def mesh_inside(ctx, tri, x, y, z, margin=0.0, want_dist=False, stream=None):
    """sbp_mesh_inside: (uint8 flags, distances or None) for the points (x, y, z)."""
    _need(tri, name="tri")
    N = x.numel()
    _exactly(_need(y, name="y"), N, "y")
    _exactly(_need(z, name="z"), N, "z")
    flags = torch.empty(N, dtype=torch.uint8, device=x.device)
    dist = torch.empty(N, dtype=torch.float32, device=x.device) if want_dist else None
    check(lib().sbp_mesh_inside(ctx.ptr, _p(tri), int(tri.numel() // 9), _p(_need(x, name="x")),
                                _p(_need(y, name="y")), _p(_need(z, name="z")), int(N), float(margin),
                                _p(flags), _p(dist), _stream(stream)))
    return flags, dist


def init_cloud(ctx, array, n, margin=2.0, a=0.1, p_lo=0.0, p_hi=0.2, seed=0, batch=1 << 20,
               device="cuda:0"):
    """n balls uniformly distributed inside the envelope (at least `margin` from
    it), p0 ~ U(p_lo, p_hi), size a; returns float32 numpy arrays."""
    dev = torch.device(device)
    tri_np = envelope_mesh(array)
    tri = torch.as_tensor(tri_np, device=dev).contiguous().view(-1)
    v = tri_np.reshape(-1, 3)
    lo, hi = v.min(0), v.max(0)
    rng = np.random.default_rng(seed)
    kept = []
    total = 0
    while total < n:
        cand = rng.uniform(lo, hi, size=(batch, 3)).astype(np.float32)
        ct = torch.as_tensor(cand, device=dev)
        flags, _ = mesh_inside(ctx, tri, ct[:, 0].contiguous(), ct[:, 1].contiguous(), ct[:, 2].contiguous(),
                               margin=margin)
        sel = cand[flags.cpu().numpy().astype(bool)]
        kept.append(sel)
        total += len(sel)
    pts = np.concatenate(kept)[:n]
    return {"x": pts[:, 0].copy(), "y": pts[:, 1].copy(), "z": pts[:, 2].copy(),
            "p0": rng.uniform(p_lo, p_hi, n).astype(np.float32), "a": np.full(n, a, np.float32)}
