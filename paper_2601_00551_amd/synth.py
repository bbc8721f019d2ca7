"""Seeded synthetic inputs: transducer arrays, phantoms, initial point clouds, noise.

This module holds no arithmetic of the reconstruction method itself; it only
draws geometry and random numbers (numpy ``default_rng``), so that the HIP
path and the FP64 oracle can be fed identical inputs.  Units: mm, us,
c = 1.5 mm/us.  The shapes follow the paper's workloads (sparse irregular
arrays of 10^2-10^3 transducers around the object, 10^5-10^6 points, 40 MHz,
section 2.1 and 2.2); the paper's own data (hand-vessel phantom, rat scans)
are not available, so these stand in for them.

Every array comes back as float32, because the ball and transducer arrays the
library works on are float32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

F32 = np.float32


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    """The generator for item ``index`` of workload ``config``: seed = 1000*config + index."""
    return np.random.default_rng(1000 * int(config) + int(index))


# --------------------------------------------------------------- arrays -----

def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _tangent_axis(n, rng):
    """A uniformly random unit vector orthogonal to each row of n."""
    r = rng.normal(size=n.shape)
    r -= np.sum(r * n, axis=-1, keepdims=True) * n
    return _unit(r)


def _rotate(v, axis, ang):
    """Rodrigues rotation of rows of v about unit rows of axis by ang (rad)."""
    c, s = np.cos(ang)[:, None], np.sin(ang)[:, None]
    return v * c + np.cross(axis, v) * s + axis * np.sum(axis * v, axis=-1, keepdims=True) * (1 - c)


def _pack_array(q, n):
    q = np.asarray(q, dtype=np.float64)
    n = _unit(np.asarray(n, dtype=np.float64))
    return {"qx": q[:, 0].astype(F32), "qy": q[:, 1].astype(F32), "qz": q[:, 2].astype(F32),
            "nx": n[:, 0].astype(F32), "ny": n[:, 1].astype(F32), "nz": n[:, 2].astype(F32)}


def hemisphere_array(n, radius, rng, tilt_deg=0.0, z_sign=-1.0):
    """n points area-uniform on the half sphere |q| = radius with z_sign*z >= 0,
    normals pointing at the centre, each tilted by |N(0, tilt_deg)| about a
    uniformly random tangent axis."""
    z = rng.uniform(0.0, 1.0, size=n) * z_sign           # area-uniform in z
    phi = rng.uniform(0.0, 2 * np.pi, size=n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    u = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    q = radius * u
    nrm = -u
    if tilt_deg > 0:
        ang = np.abs(rng.normal(0.0, np.deg2rad(tilt_deg), size=n))
        nrm = _rotate(nrm, _tangent_axis(nrm, rng), ang)
    return _pack_array(q, nrm)


def ellipsoid_array(n, semi_axes, rng, jitter=1.0):
    """n points area-uniform on the closed ellipsoid (rejection on the surface
    element), each coordinate jittered by U(-jitter, jitter); normals uniform on
    the half sphere of directions facing the centre."""
    A, Bq, C = semi_axes
    pts = []
    gmax = max(B_ * C_ for B_, C_ in ((Bq, C), (A, C), (A, Bq)))
    while sum(len(p) for p in pts) < n:
        u = _unit(rng.normal(size=(4 * n, 3)))
        # density of the map u -> (A u_x, B u_y, C u_z) relative to the sphere
        g = np.sqrt((Bq * C * u[:, 0]) ** 2 + (A * C * u[:, 1]) ** 2 + (A * Bq * u[:, 2]) ** 2)
        keep = rng.uniform(0.0, gmax, size=len(u)) < g
        pts.append(u[keep] * np.array([A, Bq, C]))
    q = np.concatenate(pts)[:n]
    q = q + rng.uniform(-jitter, jitter, size=q.shape)
    d = _unit(rng.normal(size=(n, 3)))
    inward = -_unit(q)
    d = np.where(np.sum(d * inward, axis=1, keepdims=True) < 0, -d, d)
    return _pack_array(q, d)


# ------------------------------------------------------------- phantoms -----

def _balls(x, y, z, p0, a):
    return {"x": np.asarray(x, F32), "y": np.asarray(y, F32), "z": np.asarray(z, F32),
            "p0": np.asarray(p0, F32), "a": np.asarray(a, F32)}


def polyline_phantom(rng, n_lines=3, n_vertices=4, per_line=500, half=5.0, a=0.15):
    """Vessels as polylines through n_vertices points uniform in [-half, half]^3,
    per_line balls at equal arc length, p0 ~ U(0.5, 1)."""
    xs = []
    for _ in range(n_lines):
        v = rng.uniform(-half, half, size=(n_vertices, 3))
        seg = np.linalg.norm(np.diff(v, axis=0), axis=1)
        s = np.concatenate([[0.0], np.cumsum(seg)])
        t = np.linspace(0.0, s[-1], per_line)
        xs.append(np.stack([np.interp(t, s, v[:, k]) for k in range(3)], axis=1))
    pts = np.concatenate(xs)
    p0 = rng.uniform(0.5, 1.0, size=len(pts))
    return _balls(pts[:, 0], pts[:, 1], pts[:, 2], p0, np.full(len(pts), a))


def uniform_balls(rng, n, half, a, p_lo=0.5, p_hi=1.0):
    """n balls uniform in [-half, half]^3 with p0 ~ U(p_lo, p_hi) and size a."""
    pts = rng.uniform(-half, half, size=(n, 3))
    return _balls(pts[:, 0], pts[:, 1], pts[:, 2], rng.uniform(p_lo, p_hi, size=n), np.full(n, a))


def cube_lattice(n_side, half, a, p0=0.0):
    """Cell-centred n_side^3 lattice filling [-half, half]^3."""
    h = 2.0 * half / n_side
    c = -half + h * (np.arange(n_side) + 0.5)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    n = X.size
    return _balls(X.ravel(), Y.ravel(), Z.ravel(), np.full(n, p0), np.full(n, a))


@dataclasses.dataclass
class Region:
    """Analytic reconstruction region: the cube [-half, half]^3 intersected with
    the ellipsoid of the given semi-axes (the array's ellipsoid shrunk inward)."""
    half: float
    semi_axes: tuple

    def inside(self, p):
        A, B, C = self.semi_axes
        e = (p[:, 0] / A) ** 2 + (p[:, 1] / B) ** 2 + (p[:, 2] / C) ** 2
        return (np.max(np.abs(p), axis=1) <= self.half) & (e <= 1.0)

    def lattice(self, spacing):
        n = int(np.floor(2 * self.half / spacing))
        c = -self.half + spacing * (np.arange(n) + 0.5)
        X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
        p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        return p[self.inside(p)]


def tree_phantom(rng, region: Region, spacing=0.2, a=0.1, root=(0.0, 0.0, -6.0),
                 r0=0.5, p_branch=0.7, max_depth=6, r_stop=0.1):
    """A branching tree of cylinders rasterised to balls on a `spacing` lattice.

    Root at `root` pointing +z with radius r0; each segment has length U(2, 5);
    it bifurcates with probability p_branch into children of radius
    parent * U(0.6, 0.85) turned by U(20, 60) degrees; growth stops below r_stop
    or at max_depth.  Lattice sites inside any capsule and inside the region
    become balls of size `a`; p0 ~ U(0.5, 1) per segment.
    """
    segs = []
    stack = [(np.array(root, float), np.array([0.0, 0.0, 1.0]), r0, 0)]
    while stack:
        p, d, r, depth = stack.pop()
        L = rng.uniform(2.0, 5.0)
        q = p + L * d
        segs.append((p, q, r, rng.uniform(0.5, 1.0)))
        if depth + 1 >= max_depth:
            continue
        nchild = 2 if rng.uniform() < p_branch else 1
        for _ in range(nchild):
            rc = r * rng.uniform(0.6, 0.85)
            if rc < r_stop:
                continue
            ax = _tangent_axis(d[None, :], rng)[0]
            ang = np.deg2rad(rng.uniform(20.0, 60.0))
            dc = _rotate(d[None, :], ax[None, :], np.array([ang]))[0]
            stack.append((q, _unit(dc), rc, depth + 1))
    sites = region.lattice(spacing)
    p0 = np.zeros(len(sites))
    hit = np.zeros(len(sites), dtype=bool)
    for (p, q, r, pv) in segs:
        d = q - p
        t = np.clip(((sites - p) @ d) / (d @ d), 0.0, 1.0)
        dist = np.linalg.norm(sites - (p + t[:, None] * d), axis=1)
        m = (dist <= r) & ~hit
        p0[m] = pv
        hit |= m
    pts = sites[hit]
    return _balls(pts[:, 0], pts[:, 1], pts[:, 2], p0[hit], np.full(len(pts), a))


def region_init(rng, region: Region, n, spacing=0.2, a=0.1, p_lo=0.0, p_hi=0.2, lattice=True):
    """n initial balls: lattice sites of the region drawn without replacement
    (or uniform points when lattice is False or there are fewer sites than n),
    p0 ~ U(p_lo, p_hi), size a."""
    if lattice:
        sites = region.lattice(spacing)
        if len(sites) >= n:
            idx = np.sort(rng.choice(len(sites), size=n, replace=False))
            pts = sites[idx]
            return _balls(pts[:, 0], pts[:, 1], pts[:, 2], rng.uniform(p_lo, p_hi, n), np.full(n, a))
    out = []
    while sum(len(o) for o in out) < n:
        p = rng.uniform(-region.half, region.half, size=(2 * n, 3))
        out.append(p[region.inside(p)])
    pts = np.concatenate(out)[:n]
    return _balls(pts[:, 0], pts[:, 1], pts[:, 2], rng.uniform(p_lo, p_hi, n), np.full(n, a))


def drop_near(balls, array, min_dist):
    """Remove balls closer than min_dist to any transducer (nearest-neighbour
    distances from a k-d tree over the transducer positions, FP64)."""
    from scipy.spatial import cKDTree
    p = np.stack([balls["x"], balls["y"], balls["z"]], axis=1).astype(np.float64)
    q = np.stack([array["qx"], array["qy"], array["qz"]], axis=1).astype(np.float64)
    if len(p) == 0:
        return dict(balls)
    d, _ = cKDTree(q).query(p, k=1)
    keep = d >= min_dist
    return {k: v[keep] for k, v in balls.items()}


def element_responses(n, rng, fc=2.02, bw=0.54, fc_spread=0.03, bw_spread=0.05):
    """Centre frequency (MHz) and fractional bandwidth of n transducer elements:
    the in vivo array's means (2.02 MHz, 54 %, section 2.2) with a seeded
    element-to-element spread (relative, normal; the paper reports only the
    means)."""
    f = fc * (1.0 + fc_spread * rng.standard_normal(n))
    b = bw * (1.0 + bw_spread * rng.standard_normal(n))
    return f.astype(F32), b.astype(F32)


def add_noise(y, rng, frac=0.05):
    """y + N(0, (frac * max|y|)^2), seeded."""
    y = np.asarray(y)
    sigma = frac * float(np.max(np.abs(y)))
    return (y + rng.normal(0.0, sigma, size=y.shape)).astype(y.dtype)


def concat_balls(parts):
    return {k: np.concatenate([p[k] for p in parts]).astype(F32) for k in parts[0]}


def take(balls, idx):
    return {k: np.asarray(v)[idx] for k, v in balls.items()}


# -------------------------------------------------------------- configs -----
#
# Time grids: c = 1.5 mm/us; the base interval dt is 1 / f_s.

C = 1.5


@dataclasses.dataclass
class Workload:
    name: str
    array: dict
    gt: dict           # ground-truth balls (empty dict when the workload has none)
    init: dict         # initial / current balls
    T: int             # samples at the base rate
    dt: float          # base interval, us
    levels: tuple      # downsampling factors of the schedule, coarse to fine
    a_init: float


def tiny_config(seed_index=0) -> Workload:
    """Plain method, tiny: 64 transducers on a 15 mm hemispherical cap, normals
    toward the centre tilted by |N(0, 10 deg)|; three polyline vessels of 500
    balls (a = 0.15 mm) in a 10 mm cube; 512 samples at 20 MHz; 16^3 lattice init."""
    rng = rng_for(1, seed_index)
    arr = hemisphere_array(64, 15.0, rng, tilt_deg=10.0)
    gt = polyline_phantom(rng)
    init = cube_lattice(16, 5.0, 0.15)
    init["p0"] = rng.uniform(0.0, 0.2, size=len(init["x"])).astype(F32)
    return Workload("tiny-cap64-poly1500-T512-20MHz", arr, gt, init, 512, 0.05, (1,), 0.15)


def conformal_config(seed_index=0, n_init=200_000) -> Workload:
    """Irregular conformal array: 512 transducers on a jittered ellipsoid
    (20/15/10 mm, jitter 1 mm) with random inward-facing normals; branching-tree
    phantom (radii 0.1-0.5 mm) on a 0.2 mm lattice in a 20 mm cube; n_init
    lattice sites as the initial cloud; 2048 samples at 40 MHz; levels 4, 2, 1."""
    rng = rng_for(2, seed_index)
    arr = ellipsoid_array(512, (20.0, 15.0, 10.0), rng, jitter=1.0)
    region = Region(10.0, (18.0, 13.0, 8.0))
    gt = drop_near(tree_phantom(rng, region), arr, 1.5)
    init = drop_near(region_init(rng, region, n_init), arr, 1.5)
    return Workload("conformal-ell512-tree-T2048-40MHz", arr, gt, init, 2048, 0.025, (4, 2, 1), 0.1)


def large_config(n_balls=2_000_000, n_det=1024, seed_index=0) -> Workload:
    """Large forward+adjoint: 1024 transducers on a 45 mm hemispherical cap
    around a 30 mm cube, normals toward the centre; 2M balls uniform in the cube
    (a = 0.15 mm, p0 ~ U(0.5, 1)); 4096 samples at 40 MHz."""
    rng = rng_for(3, seed_index)
    arr = hemisphere_array(n_det, 45.0, rng)
    balls = uniform_balls(rng, n_balls, 15.0, 0.15)
    return Workload("large-cap1024-uniform2M-T4096-40MHz", arr, {}, balls, 4096, 0.025, (1,), 0.15)


def batched_frames(base: Workload, n_frames=16, seed_index=0, lo=100_000, hi=2_000_000):
    """Time-resolved frames from the conformal workload: the phantom shifted by a
    vector uniform in the 1 mm ball and p0 scaled by U(0.8, 1.2) per frame; the
    initial cloud size per frame is log-uniform in [lo, hi]."""
    rng = rng_for(4, seed_index)
    region = Region(10.0, (18.0, 13.0, 8.0))
    gts, inits = [], []
    for _ in range(n_frames):
        v = _unit(rng.normal(size=(1, 3)))[0] * rng.uniform() ** (1 / 3)
        g = dict(base.gt)
        g = {k: np.asarray(val).copy() for k, val in g.items()}
        g["x"] = (g["x"] + v[0]).astype(F32)
        g["y"] = (g["y"] + v[1]).astype(F32)
        g["z"] = (g["z"] + v[2]).astype(F32)
        g["p0"] = (g["p0"] * rng.uniform(0.8, 1.2)).astype(F32)
        gts.append(g)
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        inits.append(drop_near(region_init(rng, region, n, lattice=False), base.array, 1.5))
    return gts, inits
