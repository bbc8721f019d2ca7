"""Pins of the FP64 oracle against facts the physics and mathematics fix.

None of these re-type the oracle's closed form: the forward model is checked
against a brute-force Kirchhoff spherical-mean quadrature of the initial
pressure, against a numerical integral of the textbook N-shaped pulse, against
invariances of the wave equation, and the gradients against finite differences
of the value-only forward.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import Time, UNIFORM, GAUSS, OMNI, COS, BIN, POINT


def one_ball(x=0.0, y=0.0, z=0.0, p0=1.0, a=0.15):
    return {k: np.array([v], dtype=np.float64) for k, v in
            zip(oracle.PARAMS, (x, y, z, p0, a))}


def dets(q, n):
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    n = np.asarray(n, dtype=np.float64).reshape(-1, 3)
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    return {"qx": q[:, 0], "qy": q[:, 1], "qz": q[:, 2], "nx": n[:, 0], "ny": n[:, 1], "nz": n[:, 2]}


def random_setup(rng, nb=5, nd=6, a=0.15, R=8.0, half=1.5):
    """Generic (non-lattice) small geometry: balls near the origin, detectors on
    a sphere of radius ~R with normals roughly toward the centre."""
    b = {"x": rng.uniform(-half, half, nb), "y": rng.uniform(-half, half, nb),
         "z": rng.uniform(-half, half, nb), "p0": rng.uniform(0.5, 1.0, nb),
         "a": a * rng.uniform(0.8, 1.2, nb)}
    u = rng.normal(size=(nd, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q = u * R * rng.uniform(0.95, 1.05, (nd, 1))
    n = -u + 0.3 * rng.normal(size=(nd, 3))
    return b, dets(q, n)


# ---------------------------------------------------------------- Kirchhoff --

def spherical_mean(fprof, rho, r, R):
    """Mean of a radial profile fprof(s) (support s < R) over the sphere of
    radius r centred at distance rho from the profile's centre, by adaptive
    quadrature over the polar angle."""
    if r == 0.0:
        return fprof(rho)
    pts = []
    cth = (rho * rho + r * r - R * R) / (2 * rho * r)
    if -1 < cth < 1:
        pts.append(math.acos(cth))

    def integrand(th):
        s = math.sqrt(max(rho * rho + r * r - 2 * rho * r * math.cos(th), 0.0))
        return fprof(s) * math.sin(th)

    val, _ = integrate.quad(integrand, 0.0, math.pi, points=pts or None, epsabs=1e-14,
                            epsrel=1e-12, limit=400)
    return 0.5 * val


@pytest.mark.parametrize("profile", [UNIFORM, GAUSS])
def test_bin_signal_equals_kirchhoff_spherical_means(profile):
    """Bin mean over [tau_n, tau_{n+1}) = ([t M_ct[f]] at tau_{n+1} minus at tau_n) / dt
    (Poisson-Kirchhoff: p = d/dt (t M_ct[f]) for zero initial velocity)."""
    a, K, c, dt = 0.15, 5.0, 1.5, 0.025
    R = a if profile == UNIFORM else K * a
    p0 = 0.7
    if profile == UNIFORM:
        fprof = lambda s: p0 if s < a else 0.0
    else:
        fprof = lambda s: p0 * math.exp(-s * s / (2 * a * a)) if s < K * a else 0.0
    b = one_ball(0.1, -0.2, 0.05, p0, a)
    rng = np.random.default_rng(7)
    u = rng.normal(size=(4, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q = u * np.array([[3.1], [4.37], [5.93], [7.211]])
    arr = dets(q, -u)
    T = 400
    tm = Time(c=c, dt=dt, T=T, profile=profile, directivity=OMNI, K=K)
    y = oracle.simulate(b, arr, tm)
    checked = 0
    for d in range(4):
        rho = float(np.linalg.norm(q[d] - np.array([0.1, -0.2, 0.05])))
        n_lo = int((rho - R) / (c * dt)) - 2
        n_hi = int((rho + R) / (c * dt)) + 2
        ref = np.zeros(T)
        tM = [tau * spherical_mean(fprof, rho, c * tau, R) for tau in
              (dt * np.arange(n_lo, n_hi + 2))]
        for j, n in enumerate(range(n_lo, n_hi + 1)):
            ref[n] = (tM[j + 1] - tM[j]) / dt
        assert np.max(np.abs(y[d] - ref)) <= 1e-9 * np.max(np.abs(ref))
        # outside the window everything is exactly zero
        mask = np.ones(T, bool)
        mask[n_lo:n_hi + 1] = False
        assert np.all(y[d][mask] == 0.0)
        checked += 1
    assert checked == 4


def test_gauss_truncation_error_below_bound():
    """K = 5 truncation vs the untruncated Gaussian (Kirchhoff of the full profile)."""
    a, c, dt, p0 = 0.12, 1.5, 0.025, 1.0
    b = one_ball(0, 0, 0, p0, a)
    arr = dets([[0, 0, 6.013]], [[0, 0, -1]])
    T = 300
    tm = Time(c=c, dt=dt, T=T, profile=GAUSS, directivity=OMNI, K=5.0)
    y = oracle.simulate(b, arr, tm)[0]
    rho = 6.013
    full = lambda s: p0 * math.exp(-s * s / (2 * a * a))
    taus = dt * np.arange(T + 1)
    tM = np.array([t * spherical_mean(full, rho, c * t, 50 * a) for t in taus])
    ref = np.diff(tM) / dt
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert rel < 1e-5


def test_uniform_point_and_bin_match_textbook_n_pulse():
    """UNIFORM sphere: the textbook N-shaped pulse p = p0 (rho - ct) / (2 rho) for
    |rho - ct| <= a.  POINT samples it; BIN is its exact bin average, checked by
    Gauss-Legendre quadrature split at the pulse edges (exact on linear pieces)."""
    a, c, dt, p0 = 0.15, 1.5, 0.05, 0.8
    rho = 9.8731
    b = one_ball(0, 0, 0, p0, a)
    arr = dets([[rho, 0, 0]], [[-1, 0, 0]])
    T = 200
    npulse = lambda t: p0 * (rho - c * t) / (2 * rho) if abs(rho - c * t) <= a else 0.0
    yp = oracle.simulate(b, arr, Time(c=c, dt=dt, T=T, profile=UNIFORM, directivity=OMNI,
                                      sampling=POINT))[0]
    refp = np.array([npulse(n * dt) for n in range(T)])
    np.testing.assert_allclose(yp, refp, rtol=0, atol=1e-15)
    yb = oracle.simulate(b, arr, Time(c=c, dt=dt, T=T, profile=UNIFORM, directivity=OMNI))[0]
    xg, wg = np.polynomial.legendre.leggauss(4)
    edges = sorted({(rho - a) / c, (rho + a) / c})
    refb = np.zeros(T)
    for n in range(T):
        lo, hi = n * dt, (n + 1) * dt
        cuts = [lo] + [e for e in edges if lo < e < hi] + [hi]
        s = 0.0
        for l, h in zip(cuts[:-1], cuts[1:]):
            tt = 0.5 * (h - l) * xg + 0.5 * (h + l)
            s += 0.5 * (h - l) * sum(w * npulse(t) for w, t in zip(wg, tt))
        refb[n] = s / dt
    assert np.max(np.abs(yb - refb)) <= 1e-13
    # the bins fully inside the pulse equal the textbook value at the bin centre
    inside = [n for n in range(T) if abs(rho - c * n * dt) < a and abs(rho - c * (n + 1) * dt) < a]
    assert inside
    for n in inside:
        assert abs(yb[n] - npulse((n + 0.5) * dt)) < 1e-14


# --------------------------------------------------------------- invariants --

@pytest.mark.parametrize("profile", [UNIFORM, GAUSS])
def test_superposition_and_linearity(profile):
    rng = np.random.default_rng(11)
    b, arr = random_setup(rng, nb=7, nd=5)
    tm = Time(T=900, profile=profile, directivity=COS)
    y = oracle.simulate(b, arr, tm)
    A = {k: v[:3] for k, v in b.items()}
    Bb = {k: v[3:] for k, v in b.items()}
    np.testing.assert_allclose(oracle.simulate(A, arr, tm) + oracle.simulate(Bb, arr, tm), y,
                               rtol=0, atol=1e-14 * np.max(np.abs(y)))
    lam = 2.75
    b2 = dict(b)
    b2["p0"] = lam * b["p0"]
    np.testing.assert_allclose(oracle.simulate(b2, arr, tm), lam * y, rtol=0,
                               atol=1e-14 * np.max(np.abs(y)))


def _rot(rng):
    qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(qm) < 0:
        qm[:, 0] *= -1
    return qm


@pytest.mark.parametrize("profile", [UNIFORM, GAUSS])
def test_rigid_motion_invariance(profile):
    """Rotating and translating balls, transducer positions and normals together
    leaves every trace unchanged (COS directivity included)."""
    rng = np.random.default_rng(3)
    b, arr = random_setup(rng, nb=6, nd=5)
    tm = Time(T=900, profile=profile, directivity=COS)
    y = oracle.simulate(b, arr, tm)
    Rm, t = _rot(rng), rng.normal(size=3) * 2
    P = np.stack([b["x"], b["y"], b["z"]], 1) @ Rm.T + t
    Q = np.stack([arr["qx"], arr["qy"], arr["qz"]], 1) @ Rm.T + t
    N = np.stack([arr["nx"], arr["ny"], arr["nz"]], 1) @ Rm.T
    b2 = dict(b, x=P[:, 0], y=P[:, 1], z=P[:, 2])
    arr2 = dets(Q, N)
    y2 = oracle.simulate(b2, arr2, tm)
    assert np.max(np.abs(y2 - y)) <= 1e-10 * np.max(np.abs(y))


def test_omni_rotation_about_ball_centre():
    """OMNI: moving a transducer anywhere on a sphere about a single ball's centre
    leaves its trace unchanged."""
    rng = np.random.default_rng(5)
    ctr = np.array([0.3, -0.4, 0.2])
    b = one_ball(*ctr, 0.9, 0.13)
    u = rng.normal(size=(6, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    arr = dets(ctr + 7.123 * u, -u)
    y = oracle.simulate(b, arr, Time(T=600, profile=GAUSS, directivity=OMNI))
    for d in range(1, 6):
        assert np.max(np.abs(y[d] - y[0])) <= 1e-12 * np.max(np.abs(y[0]))


@pytest.mark.parametrize("profile", [UNIFORM, GAUSS])
def test_pulse_shift_and_spherical_spreading(profile):
    """Moving a ball away from the transducer by k*c*dt along e_hat delays the
    trace by k bins and scales it by rho / (rho + delta)."""
    c, dt = 1.5, 0.025
    rho = 8.43157
    tm = Time(c=c, dt=dt, T=800, profile=profile, directivity=OMNI)
    arr = dets([[0, 0, 0]], [[1, 0, 0]])
    y0 = oracle.simulate(one_ball(rho, 0, 0, 1.0, 0.12), arr, tm)[0]
    k = 37
    delta = k * c * dt
    y1 = oracle.simulate(one_ball(rho + delta, 0, 0, 1.0, 0.12), arr, tm)[0]
    ref = np.zeros_like(y0)
    ref[k:] = y0[:-k] * rho / (rho + delta)
    assert np.max(np.abs(y1 - ref)) <= 1e-12 * np.max(np.abs(y0))


def test_cos_directivity_scaling():
    """COS: a normal along e_hat gives the OMNI trace; tilting it by theta scales
    the trace by cos(theta); a normal facing away gives zero."""
    b = one_ball(0.0, 0.0, 7.77, 1.0, 0.15)
    tmo = Time(T=800, profile=GAUSS, directivity=OMNI)
    tmc = Time(T=800, profile=GAUSS, directivity=COS)
    base = oracle.simulate(b, dets([[0, 0, 0]], [[0, 0, 1]]), tmo)[0]
    for th in (0.0, 0.4, 1.1, 1.5):
        arr = dets([[0, 0, 0]], [[math.sin(th), 0, math.cos(th)]])
        y = oracle.simulate(b, arr, tmc)[0]
        np.testing.assert_allclose(y, math.cos(th) * base, rtol=0, atol=1e-13)
    away = oracle.simulate(b, dets([[0, 0, 0]], [[0.2, 0, -1]]), tmc)[0]
    assert np.all(away == 0.0)


@pytest.mark.parametrize("profile", [UNIFORM, GAUSS])
def test_zero_sum(profile):
    """A pulse fully inside the record integrates to zero over time."""
    rng = np.random.default_rng(2)
    b, arr = random_setup(rng, nb=4, nd=3)
    y = oracle.simulate(b, arr, Time(T=1000, profile=profile, directivity=COS))
    assert np.max(np.abs(y.sum(axis=1))) <= 1e-13 * np.max(np.abs(y))


@pytest.mark.parametrize("profile", [UNIFORM, GAUSS])
@pytest.mark.parametrize("f", [2, 4, 16])
def test_pyramid_identity(profile, f):
    """Bin averaging: Downsample_f(Sim(dt, T)) = Sim(f dt, floor(T/f))."""
    rng = np.random.default_rng(9)
    b, arr = random_setup(rng, nb=5, nd=4)
    T = 1003
    y = oracle.simulate(b, arr, Time(T=T, f=1, profile=profile, directivity=COS))
    yk = oracle.simulate(b, arr, Time(T=T // f, f=f, profile=profile, directivity=COS))
    yd = oracle.downsample(y, f)
    assert yd.shape == yk.shape
    assert np.max(np.abs(yd - yk)) <= 1e-15 * max(1.0, np.max(np.abs(y)))


@pytest.mark.parametrize("f", [2, 4, 16])
def test_point_pyramid_is_decimation(f):
    """Point sampling: sample n f of Sim(dt, T) is taken at t0 + n f dt, the
    time of sample n of Sim(f dt, floor(T/f)), so Decimate_f pairs with POINT
    as Downsample_f pairs with BIN (equal up to the rounding of the sample
    times)."""
    rng = np.random.default_rng(19)
    b, arr = random_setup(rng, nb=5, nd=4)
    T = 1003
    tm1 = Time(T=T, f=1, t0=0.3, profile=GAUSS, directivity=COS, sampling=POINT)
    tmk = Time(T=T // f, f=f, t0=0.3, profile=GAUSS, directivity=COS, sampling=POINT)
    y = oracle.simulate(b, arr, tm1)
    yd = oracle.decimate(y, f)
    yk = oracle.simulate(b, arr, tmk)
    assert yd.shape == yk.shape == (4, T // f)
    assert np.count_nonzero(yk) > 20
    assert np.max(np.abs(yd - yk)) <= 1e-12 * np.max(np.abs(y))
    # and by its definition: every f-th sample, starting at sample 0
    np.testing.assert_array_equal(yd, np.stack([y[:, n * f] for n in range(T // f)], axis=1))


def test_gauss_point_equals_kirchhoff_derivative():
    """POINT under the truncated Gaussian: the value at tau_n is the Poisson-
    Kirchhoff pressure d/dt (t M_ct[f]) at t = tau_n, here by a fourth-order
    central difference of the quadrature (samples within a few steps of the
    truncation edges, where the pressure jumps, are left out)."""
    a, K, c, dt, p0 = 0.15, 5.0, 1.5, 0.025, 0.7
    R = K * a
    fprof = lambda s: p0 * math.exp(-s * s / (2 * a * a)) if s < R else 0.0
    b = one_ball(0.1, -0.2, 0.05, p0, a)
    q = np.array([[0.1, -0.2, 0.05 + 4.3717], [0.1 + 5.2209, -0.2, 0.05]])
    arr = dets(q, [[0, 0, -1], [-1, 0, 0]])
    T = 400
    y = oracle.simulate(b, arr, Time(c=c, dt=dt, T=T, profile=GAUSS, directivity=OMNI, K=K,
                                     sampling=POINT))
    h = 2e-3
    F = lambda t: t * spherical_mean(fprof, rho, c * t, R)
    checked = 0
    for d in range(2):
        rho = float(np.linalg.norm(q[d] - np.array([0.1, -0.2, 0.05])))
        edges = ((rho - R) / c, (rho + R) / c)
        ref = np.zeros(T)
        for n in range(T):
            tau = n * dt
            if not (edges[0] < tau < edges[1]):
                continue
            if min(abs(tau - e) for e in edges) < 3 * h:
                ref[n] = y[d, n]      # left out: the difference straddles the jump
                continue
            ref[n] = (-F(tau + 2 * h) + 8 * F(tau + h) - 8 * F(tau - h) + F(tau - 2 * h)) / (12 * h)
            checked += 1
        assert np.max(np.abs(y[d] - ref)) <= 1e-6 * np.max(np.abs(ref)), d
    assert checked > 70


def test_near_field_and_empty():
    arr = dets([[0, 0, 0]], [[0, 0, 1]])
    tm = Time(T=100, profile=GAUSS, directivity=OMNI)
    # transducer inside the support (rho <= K a) contributes nothing
    y = oracle.simulate(one_ball(0, 0, 0.7, 1.0, 0.15), arr, tm)
    assert np.all(y == 0.0)
    empty = {k: np.zeros(0) for k in oracle.PARAMS}
    assert np.all(oracle.simulate(empty, arr, tm) == 0.0)


def test_record_clipping():
    """A pulse straddling the end of the record keeps its in-record bins unchanged."""
    b = one_ball(0, 0, 0, 1.0, 0.15)
    arr = dets([[0, 0, 5.0]], [[0, 0, -1]])
    full = oracle.simulate(b, arr, Time(T=300, profile=GAUSS, directivity=OMNI))[0]
    nz = np.nonzero(full)[0]
    cut = int(nz.mean())
    part = oracle.simulate(b, arr, Time(T=cut, profile=GAUSS, directivity=OMNI))[0]
    np.testing.assert_array_equal(part, full[:cut])


# ---------------------------------------------------------------- gradients --

def _fd_vjp(b, arr, tm, v, h_rel=1e-6):
    out = {}
    for k in oracle.PARAMS:
        g = np.zeros(len(b["x"]))
        for i in range(len(b["x"])):
            scale = 1.0 if k in ("x", "y", "z") else abs(b[k][i])
            h = h_rel * scale
            bp = {kk: vv.copy() for kk, vv in b.items()}
            bm = {kk: vv.copy() for kk, vv in b.items()}
            bp[k][i] += h
            bm[k][i] -= h
            g[i] = np.sum(v * (oracle.simulate(bp, arr, tm) - oracle.simulate(bm, arr, tm))) / (2 * h)
        out[k] = g
    return out


@pytest.mark.parametrize("profile,directivity,sampling", [
    (GAUSS, COS, BIN), (UNIFORM, COS, BIN), (GAUSS, OMNI, BIN), (GAUSS, COS, POINT), (GAUSS, OMNI, POINT)])
def test_vjp_matches_finite_differences(profile, directivity, sampling):
    rng = np.random.default_rng(21 + profile + 2 * directivity + 4 * sampling)
    b, arr = random_setup(rng, nb=4, nd=5)
    tm = Time(T=700, f=1, profile=profile, directivity=directivity, sampling=sampling)
    v = rng.normal(size=(5, tm.T))
    g = oracle.vjp(b, arr, tm, v)
    fd = _fd_vjp(b, arr, tm, v)
    for k in oracle.PARAMS:
        den = np.max(np.abs(fd[k])) + 1e-300
        assert np.max(np.abs(g[k] - fd[k])) / den < 2e-6, (k, g[k], fd[k])


def test_vjp_value_part_matches_forward():
    """Contracting with a one-hot cotangent recovers forward values through dp0
    (the bin value is linear in p0: y = p0 * dy/dp0)."""
    rng = np.random.default_rng(4)
    b, arr = random_setup(rng, nb=1, nd=3)
    tm = Time(T=700, profile=GAUSS, directivity=COS)
    y = oracle.simulate(b, arr, tm)
    d, n = np.unravel_index(np.argmax(np.abs(y)), y.shape)
    v = np.zeros_like(y)
    v[d, n] = 1.0
    g = oracle.vjp(b, arr, tm, v)
    assert abs(g["p0"][0] * b["p0"][0] - y[d, n]) <= 1e-14 * abs(y[d, n])


def test_vjp_subset_indices():
    rng = np.random.default_rng(8)
    b, arr = random_setup(rng, nb=6, nd=3)
    tm = Time(T=700, profile=GAUSS, directivity=COS)
    v = rng.normal(size=(3, tm.T))
    full = oracle.vjp(b, arr, tm, v)
    sub = oracle.vjp(b, arr, tm, v, ball_idx=[4, 1])
    for k in oracle.PARAMS:
        np.testing.assert_array_equal(sub[k], full[k][[4, 1]])


# ------------------------------------------------------------------- filter --

def test_filter_equals_matched_filter_and_plants():
    """At p0 = 0 the gradient is g_i = -2 <y_ref, h_i> with h_i ball i's unit-p0
    trace; a ball planted in y_ref is kept, a ball no transducer sees is dropped."""
    rng = np.random.default_rng(31)
    b, arr = random_setup(rng, nb=6, nd=5)
    # ball 5 sits far behind every transducer's normal: invisible under COS
    tm = Time(T=900, profile=GAUSS, directivity=COS)
    y_ref = rng.normal(size=(5, tm.T)) * 0.01
    keep, g, out = oracle.filter_zero_grad(b, arr, tm, y_ref)
    for i in range(6):
        hb = {k: v[i:i + 1].copy() for k, v in b.items()}
        hb["p0"][:] = 1.0
        h = oracle.simulate(hb, arr, tm)
        assert abs(g[i] - (-2.0 * np.sum(y_ref * h))) <= 1e-12 * max(1e-30, np.sum(np.abs(y_ref * h)))
    np.testing.assert_array_equal(keep, g < 0)
    np.testing.assert_array_equal(out["p0"], b["p0"][keep])
    # planted ball
    j = 2
    hb = {k: v[j:j + 1].copy() for k, v in b.items()}
    hb["p0"][:] = 1.0
    hj = oracle.simulate(hb, arr, tm)
    keep2, g2, _ = oracle.filter_zero_grad(b, arr, tm, hj)
    assert g2[j] == pytest.approx(-2.0 * np.sum(hj * hj), rel=1e-12)
    assert keep2[j]
    # invisible ball: every transducer faces away -> g == 0 -> removed (strict), kept (<=)
    arr_away = dict(arr)
    for k in ("nx", "ny", "nz"):
        arr_away[k] = -np.array([arr["q" + k[1]][d] for d in range(5)])
    arr_away = dets(np.stack([arr["qx"], arr["qy"], arr["qz"]], 1),
                    np.stack([arr["qx"], arr["qy"], arr["qz"]], 1))  # normals point outward
    keep3, g3, _ = oracle.filter_zero_grad(b, arr_away, tm, y_ref)
    assert np.all(g3 == 0.0) and not np.any(keep3)
    keep4, _, _ = oracle.filter_zero_grad(b, arr_away, tm, y_ref, strict=False)
    assert np.all(keep4)


# ---------------------------------------------------- library-routine pins --

def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 8):
        g = rng.normal(size=50)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = oracle.adam_step(p, g, m, v, step, 0.01)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_softplus_matches_torch():
    import torch
    x = np.linspace(-30, 30, 601)
    np.testing.assert_allclose(oracle.softplus(x),
                               torch.nn.functional.softplus(torch.tensor(x), threshold=1e9).numpy(),
                               rtol=1e-14, atol=1e-300)
    a = np.linspace(0.01, 3, 50)
    np.testing.assert_allclose(oracle.softplus(oracle.softplus_inv(a)), a, rtol=1e-13)
    xs = np.linspace(-5, 5, 11)
    t = torch.tensor(xs, requires_grad=True)
    torch.nn.functional.softplus(t).sum().backward()
    np.testing.assert_allclose(oracle.sigmoid(xs), t.grad.numpy(), rtol=1e-14)


def test_downsample_matches_avg_pool():
    import torch
    rng = np.random.default_rng(0)
    y = rng.normal(size=(3, 4, 1001))
    for f in (1, 2, 4, 16):
        ref = torch.nn.functional.avg_pool1d(torch.tensor(y).reshape(12, 1, 1001), f, f).reshape(3, 4, -1)
        np.testing.assert_allclose(oracle.downsample(y, f), ref.numpy(), rtol=1e-14, atol=1e-15)


def test_residual_loss_sum():
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=(4, 9)), rng.normal(size=(4, 9))
    L, v = oracle.residual_loss(a, b)
    assert L == pytest.approx(float(((a - b) ** 2).sum()), rel=1e-15)
    np.testing.assert_allclose(v, 2 * (a - b))


def _grow_scene():
    """Eight hand-made balls (one frame) for the growth pins.

    index  p0    a     grad r        fate (rule below)
      0    0.9   0.2   (3, 0, 4)     candidate, |g| = 5
      1    0.01  0.2   (9, 9, 9)     destroyed: p0 < 0.05 * 0.9
      2    0.8   0.5   (0, -2, 1)    split along y (a > 0.4)
      3    0.7   0.2   (0, 0, 0)     candidate, |g| = 0
      4    0.6   0.2   (0, 6, 8)     candidate, |g| = 10
      5    0.5   0.01  (1, 1, 1)     destroyed: a < 0.02
      6    0.4   0.2   (5, 0, 0)     candidate, |g| = 5 (ties with 0)
      7    0.3   0.2   (1, 0, 0)     candidate, |g| = 1
    """
    b = {"x": np.arange(8, dtype=np.float64), "y": 10.0 + np.arange(8), "z": -np.arange(8, dtype=np.float64),
         "p0": np.array([0.9, 0.01, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3], np.float32),
         "a": np.array([0.2, 0.2, 0.5, 0.2, 0.2, 0.01, 0.2, 0.2], np.float32)}
    g = np.array([[3, 0, 4], [9, 9, 9], [0, -2, 1], [0, 0, 0], [0, 6, 8], [1, 1, 1], [5, 0, 0], [1, 0, 0]],
                 np.float32)
    grads = {"x": g[:, 0], "y": g[:, 1], "z": g[:, 2], "p0": np.zeros(8, np.float32), "a": np.zeros(8, np.float32)}
    return b, grads


def test_growth_duplicates_by_hand():
    """Five candidates (0, 3, 4, 6, 7); dup_frac 0.4 gives floor(2.0000000298) =
    2 clones: ball 4 (|g| = 10) and, of the tie 0 / 6 at |g| = 5, the lower
    index 0.  Output: survivors in input order with ball 2 replaced by its two
    children, then the clones in input order (0, then 4), each moved
    dup_offset * a = 0.1 against its gradient direction."""
    b, g = _grow_scene()
    rule = oracle.GrowthRule(destroy_frac=0.05, a_min=0.02, a_split=0.4, dup_frac=0.4, dup_offset=0.5)
    out, off, born, src = oracle.grow(b, g, rule)
    assert list(src) == [0, 2, 2, 3, 4, 6, 7, 0, 4]
    assert list(born) == [False, True, True, False, False, False, False, True, True]
    assert list(off) == [0, 9]
    # split of ball 2 along y (|g_y| = 2 is the largest): children at y -/+ a/2
    np.testing.assert_allclose(out["y"][1:3], [12.0 - 0.25, 12.0 + 0.25], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["x"][1:3], [2.0, 2.0], rtol=0, atol=0)
    np.testing.assert_allclose(out["a"][1:3], 0.5 / 2.0 ** (1.0 / 3.0), rtol=1e-15)
    # clone of ball 0: (0, 10, 0) - 0.5 * 0.2 * (3, 0, 4) / 5
    a0 = float(np.float32(0.2))
    np.testing.assert_allclose([out["x"][7], out["y"][7], out["z"][7]],
                               [-0.5 * a0 * 0.6, 10.0, -0.5 * a0 * 0.8], rtol=0, atol=1e-12)
    # clone of ball 4: (4, 14, -4) - 0.5 * 0.2 * (0, 6, 8) / 10
    np.testing.assert_allclose([out["x"][8], out["y"][8], out["z"][8]],
                               [4.0, 14.0 - 0.5 * a0 * 0.6, -4.0 - 0.5 * a0 * 0.8], rtol=0, atol=1e-12)
    assert out["p0"][7] == np.float32(0.9) and out["a"][8] == np.float32(0.2)


def test_growth_zero_gradient_clones_sit_on_their_ball():
    """With every gradient zero all keys tie: the clones go to the lowest
    candidate indices and sit exactly on their balls."""
    b, g = _grow_scene()
    g = {k: np.zeros(8, np.float32) for k in g}
    # candidates 0, 2 (not split: a_split above every a), 3, 4, 6, 7; k = 3
    rule = oracle.GrowthRule(destroy_frac=0.05, a_min=0.02, a_split=1.0, dup_frac=0.5, dup_offset=0.5)
    out, off, born, src = oracle.grow(b, g, rule)
    assert list(src) == [0, 2, 3, 4, 6, 7, 0, 2, 3]
    for ax in ("x", "y", "z"):
        np.testing.assert_array_equal(out[ax][6:], np.asarray(b[ax], np.float64)[[0, 2, 3]])


def _frac_scene():
    rng = np.random.default_rng(5)
    n = 10
    b = {"x": rng.normal(size=n).astype(np.float32), "y": rng.normal(size=n).astype(np.float32),
         "z": rng.normal(size=n).astype(np.float32), "p0": np.full(n, 0.5, np.float32),
         "a": np.full(n, 0.1, np.float32)}
    g = {k: rng.normal(size=n).astype(np.float32) for k in oracle.PARAMS}
    return b, g


def test_growth_clone_count_reads_dup_frac_as_its_float32_value():
    """The rule's thresholds are float32 fields: k = floor(n * dup_frac) with
    dup_frac the float32 value, taken exactly.  0.7 is 0.699999988 in float32,
    so ten candidates give 6 clones; 0.4 is 0.400000006, so five give 2."""
    b, g = _frac_scene()
    n = 10
    for frac, want in ((0.7, 6), (0.3, 3), (0.25, 2), (1.0, 10), (0.09, 0)):
        rule = oracle.GrowthRule(destroy_frac=0.0, a_min=0.0, a_split=1.0, dup_frac=frac, dup_offset=0.5)
        _, off, born, _ = oracle.grow(b, g, rule)
        assert born.sum() == want and off[-1] == n + want, (frac, born.sum())
    # destroy threshold: p0 < float32(destroy_frac * max p0), a tie at the threshold survives
    b["p0"] = np.array([1.0, 0.25, 0.2499999, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5], np.float32)
    rule = oracle.GrowthRule(destroy_frac=0.25, a_min=0.0, a_split=1.0, dup_frac=0.0, dup_offset=0.5)
    _, off, _, src = oracle.grow(b, g, rule)
    assert 1 in src and 2 not in src and off[-1] == 9


def test_growth_rule_self_consistency():
    """Growth thresholds are not given by the paper (parity unpinned): check
    counts, placement and ordering of the deterministic rule."""
    n = 40
    rng = np.random.default_rng(3)
    b = {"x": rng.normal(size=n), "y": rng.normal(size=n), "z": rng.normal(size=n),
         "p0": rng.uniform(0, 1, n).astype(np.float32), "a": rng.uniform(0.01, 0.5, n).astype(np.float32)}
    g = {k: rng.normal(size=n).astype(np.float32) for k in oracle.PARAMS}
    rule = oracle.GrowthRule(destroy_frac=0.1, a_min=0.05, a_split=0.35, dup_frac=0.25)
    out, off, born, src = oracle.grow(b, g, rule)
    p0 = b["p0"]
    alive = ~((p0 < np.float32(0.1) * p0.max()) | (b["a"] < np.float32(0.05)))
    split = alive & (b["a"] > np.float32(0.35))
    cand = alive & ~split
    k = int(np.floor(cand.sum() * 0.25))
    assert off[-1] == alive.sum() + split.sum() + k
    assert born.sum() == 2 * split.sum() + k
    # children straddle their parent along one axis at distance a/2 each way
    for i in np.nonzero(split)[0]:
        kids = np.nonzero(src == i)[0]
        assert len(kids) == 2
        d = np.array([out[ax][kids[1]] - out[ax][kids[0]] for ax in ("x", "y", "z")])
        assert np.isclose(np.abs(d).max(), b["a"][i]) and np.count_nonzero(np.abs(d) > 1e-12) == 1
        assert np.allclose(out["a"][kids], b["a"][i] / 2 ** (1 / 3))
