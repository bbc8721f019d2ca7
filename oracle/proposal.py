"""Reference of the growth-proposal inputs and outputs (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; it shares no code with the HIP library.

The learned proposal extends the growth step of section 4.1 (where new balls
appear next to existing ones): a regular grid of cells, candidate sites in
the empty cells that touch an occupied one, a 31-value feature row per site,
and the insertion of the sites the network accepts.  These are plain
definitions, written out in FP64 except where a floating-point value decides
an integer (the cell a point falls in), which is taken in FP32 as the GPU
takes it.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Grid:
    ox: float
    oy: float
    oz: float
    h: float
    nx: int
    ny: int
    nz: int


def cell_index(grid, x, y, z):
    """(i, j, k, inside) of points, with the FP32 floor((x - origin) / h)."""
    f = np.float32
    h = f(grid.h)
    i = np.floor((np.asarray(x, f) - f(grid.ox)) / h).astype(np.int64)
    j = np.floor((np.asarray(y, f) - f(grid.oy)) / h).astype(np.int64)
    k = np.floor((np.asarray(z, f) - f(grid.oz)) / h).astype(np.int64)
    inside = (i >= 0) & (j >= 0) & (k >= 0) & (i < grid.nx) & (j < grid.ny) & (k < grid.nz)
    return i, j, k, inside


def grid_mass(grid, balls):
    """mass[i, j, k] = sum of p0 over the balls whose centre lies in cell (i, j, k)."""
    i, j, k, ins = cell_index(grid, balls["x"], balls["y"], balls["z"])
    m = np.zeros((grid.nx, grid.ny, grid.nz))
    np.add.at(m, (i[ins], j[ins], k[ins]), np.asarray(balls["p0"], np.float64)[ins])
    return m


NEIGHBOURS = [(di, dj, dk) for di in (-1, 0, 1) for dj in (-1, 0, 1) for dk in (-1, 0, 1)
              if (di, dj, dk) != (0, 0, 0)]


def candidates(grid, mass, occ):
    """Flat indices (i*ny + j)*nz + k, in increasing order, of the cells with
    mass < occ that have a 26-neighbour with mass >= occ, and their centres."""
    occupied = np.asarray(mass) >= occ
    nx, ny, nz = occupied.shape
    pad = np.zeros((nx + 2, ny + 2, nz + 2), bool)
    pad[1:-1, 1:-1, 1:-1] = occupied
    near = np.zeros_like(occupied)
    for di, dj, dk in NEIGHBOURS:
        near |= pad[1 + di:1 + di + nx, 1 + dj:1 + dj + ny, 1 + dk:1 + dk + nz]
    cand = near & ~occupied
    flat = np.flatnonzero(cand.ravel())
    i, rem = np.divmod(flat, ny * nz)
    j, k = np.divmod(rem, nz)
    centre = np.stack([grid.ox + (i + 0.5) * grid.h, grid.oy + (j + 0.5) * grid.h,
                       grid.oz + (k + 0.5) * grid.h], axis=1)
    return flat, centre


def features(grid, mass, xyz, g_p0, g_r, half):
    """Feature rows [M][31]: probe back-projection, probe gradient norm, the 26
    neighbour masses and the position (each scaled as the header states)."""
    xyz = np.asarray(xyz, np.float64)
    M = xyz.shape[0]
    X = np.zeros((M, 31))
    gp = np.asarray(g_p0, np.float64)
    gn = np.linalg.norm(np.asarray(g_r, np.float64), axis=1)
    sa, sb, sc = (np.max(np.abs(gp)) if M else 0.0), (np.max(gn) if M else 0.0), np.max(np.abs(mass))
    X[:, 0] = -gp / sa if sa > 0 else 0.0
    X[:, 1] = gn / sb if sb > 0 else 0.0
    i, j, k, ins = cell_index(grid, xyz[:, 0], xyz[:, 1], xyz[:, 2])
    nx, ny, nz = mass.shape
    for q, (di, dj, dk) in enumerate(NEIGHBOURS):
        a, b, c = i + di, j + dj, k + dk
        ok = ins & (a >= 0) & (b >= 0) & (c >= 0) & (a < nx) & (b < ny) & (c < nz)
        v = np.zeros(M)
        v[ok] = mass[a[ok], b[ok], c[ok]]
        X[:, 2 + q] = v / sc if sc > 0 else 0.0
    X[:, 28:31] = xyz / half
    return X


def append(balls, sites, out, a_init, p0_scale=1.0):
    """The balls after appending the accepted sites (logit > 0) in site order,
    with p0 = max(predicted p0, 0) * p0_scale."""
    out = np.asarray(out, np.float64)
    acc = out[:, 0] > 0
    new = {"x": sites[acc, 0], "y": sites[acc, 1], "z": sites[acc, 2],
           "p0": np.maximum(out[acc, 1], 0.0) * p0_scale, "a": np.full(int(acc.sum()), float(a_init))}
    return {k: np.concatenate([np.asarray(balls[k], np.float64), new[k]]) for k in new}


def merge(balls, ball_off, sites, site_off, out, p0_scale, a_init, extra=None):
    """Per frame: the frame's balls in order, then its accepted sites in site
    order (logit > 0 and the frame's p0_scale > 0) with p0 = max(predicted p0,
    0) * p0_scale[f] and size a_init.  `extra` maps names (gradients, moments)
    to per-ball arrays carried with their balls; the new balls get zeros.
    Returns (balls, ball_off, extra) of the merged state."""
    out = np.asarray(out, np.float64)
    sites = np.asarray(sites, np.float64)
    F = len(ball_off) - 1
    keys = ("x", "y", "z", "p0", "a")
    extra = extra or {}
    nb = {k: [] for k in keys}
    ne = {k: [] for k in extra}
    off = [0]
    for f in range(F):
        lo, hi = int(ball_off[f]), int(ball_off[f + 1])
        for k in keys:
            nb[k].append(np.asarray(balls[k][lo:hi], np.float64))
        for k in extra:
            ne[k].append(np.asarray(extra[k][lo:hi], np.float64))
        s0, s1 = int(site_off[f]), int(site_off[f + 1])
        acc = (out[s0:s1, 0] > 0) & (p0_scale[f] > 0)
        n = int(acc.sum())
        nb["x"].append(sites[s0:s1, 0][acc])
        nb["y"].append(sites[s0:s1, 1][acc])
        nb["z"].append(sites[s0:s1, 2][acc])
        nb["p0"].append(np.maximum(out[s0:s1, 1][acc], 0.0) * p0_scale[f])
        nb["a"].append(np.full(n, float(a_init)))
        for k in extra:
            ne[k].append(np.zeros(n))
        off.append(off[-1] + (hi - lo) + n)
    return ({k: np.concatenate(v) for k, v in nb.items()}, np.array(off, np.int64),
            {k: np.concatenate(v) for k, v in ne.items()})
