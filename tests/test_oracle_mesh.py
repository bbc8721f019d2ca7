"""Pins of the envelope-test reference (no GPU): a cube and a tetrahedron,
whose inside and distance are known in closed form, and the convex hull of
points on an ellipsoid against the analytic ellipsoid."""
import numpy as np
import pytest

from oracle import mesh as om


def cube_mesh(lo=-1.0, hi=1.0):
    v = np.array([[x, y, z] for x in (lo, hi) for y in (lo, hi) for z in (lo, hi)], float)
    faces = [(0, 1, 3), (0, 3, 2), (4, 6, 7), (4, 7, 5), (0, 4, 5), (0, 5, 1),
             (2, 3, 7), (2, 7, 6), (0, 2, 6), (0, 6, 4), (1, 5, 7), (1, 7, 3)]
    return np.array([np.concatenate([v[a], v[b], v[c]]) for a, b, c in faces], np.float32)


def test_cube_inside_and_distance():
    tri = cube_mesh()
    rng = np.random.default_rng(0)
    p = rng.uniform(-1.5, 1.5, size=(4000, 3))
    ins = om.inside(tri, p)
    exp = np.all(np.abs(p) < 1.0, axis=1)
    band = np.min(np.abs(np.abs(p) - 1.0), axis=1) < 1e-5
    np.testing.assert_array_equal(ins[~band], exp[~band])
    d = om.distance(tri, p)
    # inside: distance to the nearest face; outside: Euclidean distance to the box
    din = np.min(1.0 - np.abs(p), axis=1)
    dout = np.linalg.norm(np.maximum(np.abs(p) - 1.0, 0.0), axis=1)
    np.testing.assert_allclose(d, np.where(exp, din, dout), rtol=1e-12, atol=1e-12)


def test_margin():
    tri = cube_mesh()
    p = np.array([[0.0, 0.0, 0.0], [0.85, 0.0, 0.0], [0.0, -0.95, 0.1], [1.2, 0, 0]])
    np.testing.assert_array_equal(om.inside(tri, p, margin=0.1), [True, True, False, False])


def test_tetrahedron_crossings():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    faces = [(0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3)]
    tri = np.array([np.concatenate([v[a], v[b], v[c]]) for a, b, c in faces], np.float32)
    p = np.array([[0.1, 0.1, 0.1], [0.4, 0.4, 0.4], [-0.5, 0.2, 0.2], [0.2, 0.2, 0.2]])
    # inside iff x, y, z > 0 and x + y + z < 1; a ray from outside enters and leaves
    np.testing.assert_array_equal(om.crossings(tri, p) % 2, [1, 0, 0, 1])
    assert om.crossings(tri, p)[2] in (0, 2)


def test_hull_of_ellipsoid_points():
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(1)
    u = rng.normal(size=(600, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q = u * [4.0, 3.0, 2.0]
    hull = ConvexHull(q)
    tri = q[hull.simplices].reshape(-1, 9)
    p = rng.uniform(-4, 4, size=(3000, 3)) * [1, 0.75, 0.5]
    e = (p[:, 0] / 4) ** 2 + (p[:, 1] / 3) ** 2 + (p[:, 2] / 2) ** 2
    ins = om.inside(tri, p)
    # the hull lies inside the ellipsoid and hugs it: agreement away from the surface
    far = np.abs(e - 1.0) > 0.15
    np.testing.assert_array_equal(ins[far], (e < 1.0)[far])
