"""Reference of the envelope test used to draw the initial cloud inside the
array (test infrastructure only; shares no code with the HIP library).

Algorithm 1 of SlingBAG Pro builds a closed polygonal envelope mesh from the
array coordinates and draws the random initial points inside it by ray
casting.  A point is inside when a ray from it crosses the mesh an odd number
of times; it is kept when it is also at least `margin` from the mesh (the
region is defined inward of the envelope).  The crossing test is taken in
FP32 (it decides an integer, and the kernel takes it in FP32); distances are
FP64.
"""
from __future__ import annotations

import numpy as np

DIRECTION = np.array([1.0, 0.7071, 0.3183], dtype=np.float32)


def crossings(tri, pts):
    """Number of triangles the ray p + t d (t > 0) crosses, per point (FP32)."""
    tri = np.asarray(tri, np.float32).reshape(-1, 3, 3)
    p = np.asarray(pts, np.float32)
    d = DIRECTION
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    e1, e2 = b - a, c - a
    h = np.cross(np.broadcast_to(d, e2.shape), e2).astype(np.float32)
    det = np.einsum("ij,ij->i", e1, h).astype(np.float32)
    count = np.zeros(len(p), np.int64)
    for k in range(len(tri)):
        if det[k] == 0:
            continue
        f = np.float32(1.0) / det[k]
        s = p - a[k]
        u = f * (s @ h[k])
        q = np.cross(s, e1[k]).astype(np.float32)
        w = f * (q @ d)
        t = f * (q @ e2[k])
        count += ((u >= 0) & (u <= 1) & (w >= 0) & (u + w <= 1) & (t > 0)).astype(np.int64)
    return count


def _seg_dist(p, a, b):
    ab = b - a
    t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(p - (a + t[:, None] * ab), axis=1)


def distance(tri, pts):
    """Distance from each point to the nearest triangle (FP64): the distance to
    the plane where the projection falls inside the triangle, else to the
    nearest edge."""
    tri = np.asarray(tri, np.float64).reshape(-1, 3, 3)
    p = np.asarray(pts, np.float64)
    best = np.full(len(p), np.inf)
    for a, b, c in tri:
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        sd = (p - a) @ n
        proj = p - sd[:, None] * n
        # barycentric sign test of the projection
        s1 = np.cross(b - a, proj - a) @ n
        s2 = np.cross(c - b, proj - b) @ n
        s3 = np.cross(a - c, proj - c) @ n
        inside = ((s1 >= 0) & (s2 >= 0) & (s3 >= 0)) | ((s1 <= 0) & (s2 <= 0) & (s3 <= 0))
        d = np.where(inside, np.abs(sd), np.minimum(np.minimum(_seg_dist(p, a, b), _seg_dist(p, b, c)),
                                                    _seg_dist(p, c, a)))
        best = np.minimum(best, d)
    return best


def inside(tri, pts, margin=0.0):
    odd = crossings(tri, pts) % 2 == 1
    if margin > 0:
        return odd & (distance(tri, pts) >= margin)
    return odd
