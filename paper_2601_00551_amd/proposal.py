"""Learned growth proposal: a BF16 MLP on the matrix cores that decides where
new balls appear and with which p0 (declared in include/sbp_mlp.h).

Section 4.1 of SlingBAG Pro grows the cloud by splitting, destroying and
duplicating balls from pressure / size thresholds.  The network adds a second
source of new balls at the same growth points: candidate sites are the empty
cells of a regular grid that touch an occupied cell; each gets a feature row
(the residual back-projected onto a unit probe ball at the site, the probe's
gradient norm, the 26 neighbour masses and the position) and the network
returns a growth logit and an initial p0.  The accepted sites are appended as
balls.  The data-fidelity loss is the judge: if the appended balls do not
lower the loss, they are removed again and only the plain rule has acted.

Training data come from reconstructions the plain method itself runs: the
features of the candidate sites at its growth points, labelled by the mass the
plain reconstruction ends up with in the candidate's cell (grow if above a
threshold; the regression target is that mass).

Every step runs in libsbp.so (feature kernels, MLP forward / loss / backward /
Adam kernels); this module marshals arguments, sequences calls and prepares
training sets.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
import json
import sys
import time

import numpy as np
import torch

from . import _abi, api, recon, synth
from ._abi import MLP_HID, MLP_IN, MLP_NPARAM, MLP_NWORK, check, lib
from .api import P0, PARAMS, XYZ, _at_least, _check_balls, _exactly, _need, _p, _stream, balls_struct

# flat FP32 parameter layout of the network (row-major [in][out], then bias)
LAYOUT = [("W1", (32, MLP_HID)), ("b1", (MLP_HID,)), ("W2", (MLP_HID, MLP_HID)), ("b2", (MLP_HID,)),
          ("W3", (MLP_HID, MLP_HID)), ("b3", (MLP_HID,)), ("W4", (MLP_HID, 2)), ("b4", (2,))]


def padded(M: int) -> int:
    return (int(M) + 63) // 64 * 64


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (the zero-padding input row 31 stays zero), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in LAYOUT:
        if name.startswith("b"):
            parts.append(np.zeros(shape))
            continue
        fan_in = MLP_IN if name == "W1" else shape[0]
        gain = 1.0 if name == "W4" else 2.0
        w = rng.normal(0.0, np.sqrt(gain / fan_in), size=shape)
        if name == "W1":
            w[MLP_IN:, :] = 0.0
        parts.append(w)
    p = np.concatenate([x.ravel() for x in parts]).astype(np.float32)
    assert p.size == MLP_NPARAM
    return p


class ProposalMLP:
    """Parameters (FP32), their BF16 working copies and Adam moments, on one device."""

    def __init__(self, ctx, device="cuda:0", seed=0, params=None):
        self.ctx = ctx
        self.dev = torch.device(device)
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        if p.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters, got {p.size}")
        self.params = torch.as_tensor(p, device=self.dev).contiguous()
        self.work = torch.empty(MLP_NWORK, dtype=torch.int16, device=self.dev)
        self.grad = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=self.dev)
        self.m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=self.dev)
        self.t = 0
        self._bufs = {}
        self.sync()

    def sync(self, stream=None):
        check(lib().sbp_mlp_sync(self.ctx.ptr, _p(self.params), _p(self.work), _stream(stream)))

    def forward(self, X, out=None, acts=None, stream=None):
        """out [M][2] = (growth logit, initial p0) for feature rows X [M][31]."""
        _need(X, name="X")
        M = X.shape[0]
        if X.dim() != 2 or X.shape[1] != MLP_IN:
            raise ValueError("X must be [M][31]")
        if out is None:
            out = torch.empty((M, 2), dtype=torch.float32, device=X.device)
        _at_least(_need(out, name="out"), 2 * M, "out")
        if acts is not None:
            _at_least(acts, (32 + 3 * MLP_HID) * padded(M), "acts")
        check(lib().sbp_mlp_forward(self.ctx.ptr, _p(self.params), _p(self.work), _p(X), M,
                                    _p(_need(out, name="out")), _p(acts), _stream(stream)))
        return out

    def _buffers(self, M):
        Mp = padded(M)
        b = self._bufs.get(Mp)
        if b is None:
            d = self.dev
            b = dict(acts=torch.empty((32 + 3 * MLP_HID) * Mp, dtype=torch.int16, device=d),
                     dacts=torch.empty(3 * MLP_HID * Mp, dtype=torch.int16, device=d),
                     dout=torch.empty(2 * Mp, dtype=torch.float32, device=d),
                     dout_t=torch.empty(16 * Mp, dtype=torch.int16, device=d),
                     loss=torch.zeros(1, dtype=torch.float64, device=d))
            self._bufs = {Mp: b}
        return b

    def loss_and_grad(self, X, yg, yp, pos_weight=1.0, stream=None):
        """Mean loss (device double) and self.grad = d loss / d params."""
        M = X.shape[0]
        b = self._buffers(M)
        out = torch.empty((M, 2), dtype=torch.float32, device=X.device)
        self.forward(X, out=out, acts=b["acts"], stream=stream)
        _at_least(_need(yg, name="yg"), M, "yg")
        _at_least(_need(yp, name="yp"), M, "yp")
        check(lib().sbp_mlp_loss(self.ctx.ptr, _p(out), _p(yg), _p(yp),
                                 M, float(pos_weight), _p(b["loss"]), _p(b["dout"]), _p(b["dout_t"]),
                                 _stream(stream)))
        check(lib().sbp_mlp_backward(self.ctx.ptr, _p(self.work), _p(b["acts"]), _p(b["dout"]),
                                     _p(b["dout_t"]), M, _p(b["dacts"]), _p(self.grad), _stream(stream)))
        return b["loss"], out

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.t += 1
        prm = api.AdamParams(lr=(lr,) * 5, beta1=beta1, beta2=beta2, eps=eps, step=self.t)
        check(lib().sbp_mlp_adam(self.ctx.ptr, _p(self.params), _p(self.grad), _p(self.m), _p(self.v),
                                 ctypes.byref(prm.struct()), _p(self.work), _stream(stream)))

    def train_step(self, X, yg, yp, pos_weight=1.0, lr=1e-3, stream=None):
        loss, _ = self.loss_and_grad(X, yg, yp, pos_weight, stream)
        self.adam(lr=lr, stream=stream)
        return loss

    def save(self, path, bf16=False):
        """Write the parameters (.npz).  bf16=True stores them rounded to
        BF16 (to nearest, ties to even) as their 16-bit patterns: the matrix
        cores read BF16 copies, so inference from the file is unchanged and
        the file is half the size."""
        p = self.params.cpu().numpy()
        if bf16:
            bits = p.view(np.uint32).astype(np.uint64)
            rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)
            np.savez_compressed(path, params_bf16=rounded)
        else:
            np.savez(path, params=p)

    @classmethod
    def load(cls, ctx, path, device="cuda:0"):
        with np.load(path) as z:
            if "params_bf16" in z:
                p = (z["params_bf16"].astype(np.uint32) << 16).view(np.float32)
            else:
                p = z["params"]
            return cls(ctx, device=device, params=p)


# ------------------------------------------------------ candidate sites --

@dataclasses.dataclass
class Grid:
    ox: float
    oy: float
    oz: float
    h: float
    nx: int
    ny: int
    nz: int

    @classmethod
    def cube(cls, half, h):
        n = int(round(2 * half / h))
        return cls(-half, -half, -half, h, n, n, n)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    def struct(self):
        return _abi.SbpGrid(self.ox, self.oy, self.oz, self.h, self.nx, self.ny, self.nz, 0)


def grid_mass(ctx, balls, ball_off, grid: Grid, B_cap=None, mass=None, stream=None):
    """sbp_grid_mass: p0 summed per cell over frame 0."""
    dev = balls["x"].device
    if mass is None:
        mass = torch.empty(grid.ncell, dtype=torch.float32, device=dev)
    cap = balls["x"].numel() if B_cap is None else int(B_cap)
    _check_balls(balls, cap)
    _exactly(_need(mass, name="mass"), grid.ncell, "mass")
    check(lib().sbp_grid_mass(ctx.ptr, ctypes.byref(balls_struct(balls)), _p(_need(ball_off, torch.int64, "ball_off")),
                              cap, ctypes.byref(grid.struct()), _p(_need(mass, name="mass")), _stream(stream)))
    return mass


def candidates(ctx, grid: Grid, mass, occ, a_probe, sites=None, stream=None):
    """sbp_candidates: (sites as a probe-ball SoA of capacity ncell, count)."""
    dev = mass.device
    if sites is None:
        sites = {k: torch.empty(grid.ncell, dtype=torch.float32, device=dev) for k in PARAMS}
    cap = sites["x"].numel()
    _check_balls(sites, cap, "sites")
    _exactly(_need(mass, name="mass"), grid.ncell, "mass")
    cnt = ctypes.c_int64()
    check(lib().sbp_candidates(ctx.ptr, ctypes.byref(grid.struct()), _p(_need(mass, name="mass")), float(occ),
                               float(a_probe), ctypes.byref(balls_struct(sites)), cap, ctypes.byref(cnt),
                               _stream(stream)))
    return sites, cnt.value


def features(ctx, grid: Grid, mass, sites, M, g, half, X=None, stream=None):
    """sbp_features: feature rows [M][31]."""
    dev = mass.device
    if X is None:
        X = torch.empty((M, MLP_IN), dtype=torch.float32, device=dev)
    _exactly(_need(mass, name="mass"), grid.ncell, "mass")
    _check_balls(sites, M, "sites")
    _check_balls({k: g[k] for k in ("x", "y", "z", "p0")}, M, "g")
    _at_least(_need(X, name="X"), M * MLP_IN, "X")
    gb = _abi.SbpBalls(_p(g["x"]), _p(g["y"]), _p(g["z"]), _p(g["p0"]), None)
    check(lib().sbp_features(ctx.ptr, ctypes.byref(grid.struct()), _p(mass), ctypes.byref(balls_struct(sites)),
                             int(M), ctypes.byref(gb), float(half), _p(_need(X, name="X")), _stream(stream)))
    return X


def append_proposals(ctx, state: api.State, sites, out, M, a_init, p0_scale=1.0, stream=None):
    """sbp_append_proposals: returns the new ball count of frame 0."""
    _check_balls(sites, M, "sites")
    _at_least(_need(out, name="out"), 2 * M, "out")
    cnt = ctypes.c_int64()
    check(lib().sbp_append_proposals(ctx.ptr, ctypes.byref(state.struct()), ctypes.byref(balls_struct(sites)),
                                     _p(_need(out, name="out")), int(M), float(a_init), float(p0_scale),
                                     ctypes.byref(cnt), _stream(stream)))
    return cnt.value


def merge_proposals(ctx, state: api.State, sites, site_off, out, p0_scale, a_init, out_state=None,
                    capacity=None, stream=None):
    """sbp_merge_proposals: a new state holding every frame's balls followed by
    its accepted sites (site_off: device int64 [F+1], p0_scale: device float [F])."""
    F = state.F
    _exactly(_need(site_off, torch.int64, "site_off"), F + 1, "site_off")
    _exactly(_need(p0_scale, name="p0_scale"), F, "p0_scale")
    M = int(site_off[-1].item())
    _check_balls(sites, M, "sites")
    if M > 0:
        _at_least(_need(out, name="out"), 2 * M, "out")
    if out_state is None:
        cap = int(capacity if capacity is not None else state.B_cap + M)
        out_state = api.State({k: np.zeros(0) for k in PARAMS}, ball_off=[0] * (F + 1), capacity=cap,
                              device=state.ball_off.device)
    cnt = ctypes.c_int64()
    check(lib().sbp_merge_proposals(ctx.ptr, ctypes.byref(state.struct()), ctypes.byref(balls_struct(sites)),
                                    _p(site_off), _p(out) if M > 0 else None, M, _p(p0_scale), float(a_init),
                                    ctypes.byref(out_state.struct()), ctypes.byref(cnt), _stream(stream)))
    return out_state, cnt.value


class FeatureBuilder:
    """Candidate sites and their features for one state, reusing its buffers."""

    def __init__(self, ctx, grid: Grid, occ=0.1, a_probe=0.1, half=10.0, device="cuda:0"):
        self.ctx, self.grid, self.occ, self.a_probe, self.half = ctx, grid, occ, a_probe, half
        dev = torch.device(device)
        self.mass = torch.empty(grid.ncell, dtype=torch.float32, device=dev)
        self.sites = {k: torch.empty(grid.ncell, dtype=torch.float32, device=dev) for k in PARAMS}
        self.g = {k: torch.empty(grid.ncell, dtype=torch.float32, device=dev) for k in PARAMS}
        self.off = torch.zeros(2, dtype=torch.int64, device=dev)

    def build(self, A, state: api.State, model: api.Model, v):
        """(M, X [M][31], sites) given v = dL/dy_sim of the current state."""
        grid_mass(self.ctx, state.balls, state.ball_off, self.grid, B_cap=state.B_cap, mass=self.mass)
        _, M = candidates(self.ctx, self.grid, self.mass, self.occ, self.a_probe, sites=self.sites)
        if M == 0:
            return 0, None, self.sites
        self.off[1] = M
        probe_model = dataclasses.replace(model, a_softplus=0)
        api.adjoint_gradients(self.ctx, A, self.sites, probe_model, v, mask=P0 | XYZ, ball_off=self.off,
                              grad=self.g, B_cap=M)
        X = features(self.ctx, self.grid, self.mass, self.sites, M, self.g, self.half)
        return M, X, self.sites


def _residual(r: recon.Recon, model, y_k, yw):
    st = r.state
    api.simulate_signals(r.ctx, r.A, st.balls, model, ball_off=st.ball_off, y=yw, B_cap=st.B_cap)
    return float(api.residual_loss(r.ctx, yw, y_k, v_out=yw).sum().item())


class FrameFeatureBuilder(FeatureBuilder):
    """Candidate sites and features of every frame of a state, back to back
    (frame f's rows from site_off[f]), for the multi-frame proposer."""

    def __init__(self, ctx, grid: Grid, occ=0.1, a_probe=0.1, half=10.0, device="cuda:0"):
        super().__init__(ctx, grid, occ, a_probe, half, device)
        self.cap = 0
        self.all_sites = self.all_g = self.X = None

    def _grow_to(self, n):
        if n <= self.cap:
            return
        dev = self.mass.device
        self.all_sites = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in PARAMS}
        self.all_g = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in PARAMS}
        self.X = torch.empty((n, MLP_IN), dtype=torch.float32, device=dev)
        self.cap = n

    def build_frames(self, A, state: api.State, model: api.Model, v):
        """(M_total, X [M_total][31], sites, site_off device [F+1]) given
        v [F][D][T] = dL/dy_sim of the current state."""
        F = state.F
        nc = self.grid.ncell
        self._grow_to(F * nc)
        probe_model = dataclasses.replace(model, a_softplus=0)
        offs = [0]
        for f in range(F):
            o = offs[-1]
            grid_mass(self.ctx, state.balls, state.ball_off[f:], self.grid, B_cap=state.B_cap, mass=self.mass)
            view = {k: self.all_sites[k][o:o + nc] for k in PARAMS}
            _, M = candidates(self.ctx, self.grid, self.mass, self.occ, self.a_probe, sites=view)
            if M > 0:
                self.off[1] = M
                gv = {k: self.all_g[k][o:o + M] for k in PARAMS}
                api.adjoint_gradients(self.ctx, A, {k: view[k][:M] for k in PARAMS}, probe_model,
                                      v[f:f + 1], mask=P0 | XYZ, ball_off=self.off, grad=gv, B_cap=M)
                features(self.ctx, self.grid, self.mass, view, M, gv, self.half, X=self.X[o:o + M])
            offs.append(o + M)
        site_off = torch.tensor(offs, dtype=torch.int64, device=self.mass.device)
        return offs[-1], self.X[:offs[-1]], self.all_sites, site_off


class Recorder:
    """Growth-point hook for plain runs: keeps the candidates' features."""

    def __init__(self, builder: FeatureBuilder):
        self.builder = builder
        self.events = []

    def __call__(self, r: recon.Recon, si, model, y_k, yw):
        _residual(r, model, y_k, yw)
        M, X, sites = self.builder.build(r.A, r.state, model, yw)
        if M == 0:
            return
        xyz = torch.stack([sites["x"][:M], sites["y"][:M], sites["z"][:M]], dim=1).cpu().numpy()
        self.events.append(dict(stage=si, X=X.cpu().numpy(), xyz=xyz))


class LearnedProposer:
    """Growth-point hook that appends the sites the network accepts.

    The accepted balls enter along one direction of the parameter space (their
    predicted p0 values); their common scale is the exact minimiser of the
    quadratic loss along it, alpha* = -<e, s> / <s, s> (e the current
    residual, s the signal of the appended balls at the predicted p0), taken
    from three loss evaluations: ||e||^2, ||s||^2 and ||e + s||^2.  If
    alpha* <= 0, or the loss at alpha* is not below ||e||^2 (the judge), the
    balls are removed again.
    """

    def __init__(self, mlp: ProposalMLP, builder: FeatureBuilder, a_init=0.1, judge=True,
                 max_scale=4.0, stages=None, max_per_stage=None, patience=None, reprobe_every=None):
        self.mlp, self.builder, self.a_init, self.judge = mlp, builder, a_init, judge
        self.max_scale = max_scale
        self.stages = None if stages is None else set(stages)   # stage indices it acts in
        self.max_per_stage = max_per_stage                       # growth points per stage
        # the gate: after `patience` proposals in a row that the loss judge
        # rejected, the network stays off (None: never).  With reprobe_every
        # = None the gate is per run (new_run opens it again); with a number
        # it carries over the runs of one configuration and reopens for one
        # probe every `reprobe_every` runs.
        self.patience = patience
        self.reprobe_every = reprobe_every
        self.rejected_in_a_row = 0
        self.gated = False
        self.runs = 0
        self.closed_at_run = None
        self.events = []
        self._zero = None
        self._ys = None
        self._off = None

    def new_run(self):
        """Call before each reconstruction the proposer serves."""
        self.runs += 1
        if self.reprobe_every is None:
            self.gated, self.rejected_in_a_row = False, 0
        elif self.gated and self.runs - self.closed_at_run >= self.reprobe_every:
            self.gated = False
            self.rejected_in_a_row = max(0, (self.patience or 1) - 1)   # one probe

    def __call__(self, r: recon.Recon, si, model, y_k, yw):
        if self.gated:
            return
        if self.stages is not None and si not in self.stages:
            return
        if self.max_per_stage is not None and \
                sum(e["stage"] == si and e["run"] == self.runs for e in self.events) >= self.max_per_stage:
            return
        t0 = time.perf_counter()
        ev = dict(run=self.runs, stage=si, candidates=0, accepted=0, kept=False, scale=0.0)
        self.events.append(ev)
        try:
            self._propose(r, model, y_k, yw, ev)
        finally:
            if yw.is_cuda:
                torch.cuda.synchronize(yw.device)
            ev["seconds"] = time.perf_counter() - t0
        self.rejected_in_a_row = 0 if ev["kept"] else self.rejected_in_a_row + 1
        if self.patience is not None and self.rejected_in_a_row >= self.patience:
            self.gated = True
            self.closed_at_run = self.runs
            ev["gate_closed"] = True

    def _frame_losses(self, r, model, state, y_k, yw):
        api.simulate_signals(r.ctx, r.A, state.balls, model, ball_off=state.ball_off, y=yw, B_cap=state.B_cap)
        return api.residual_loss(r.ctx, yw, y_k, v_out=yw).cpu().numpy()

    def _propose_frames(self, r, model, y_k, yw, ev):
        """Every frame at once: candidate sites and features per frame, one
        network pass over all of them, then per frame the exact line search
        along its proposals and the loss judge; the accepted proposals of all
        frames are merged into a new state (sbp_merge_proposals)."""
        st = r.state
        F = st.F
        dev = yw.device
        L0 = self._frame_losses(r, model, st, y_k, yw)          # yw = dL/dy_sim now
        ev.update(loss_before=float(L0.sum()), loss_after=float(L0.sum()))
        if not isinstance(self.builder, FrameFeatureBuilder):
            b = self.builder
            self.builder = FrameFeatureBuilder(r.ctx, b.grid, b.occ, b.a_probe, b.half, device=dev)
        M, X, sites, site_off = self.builder.build_frames(r.A, st, model, yw)
        ev["candidates"] = M
        if M == 0:
            return
        out = self.mlp.forward(X)
        ones = torch.ones(F, dtype=torch.float32, device=dev)
        empty = api.State({k: np.zeros(0) for k in PARAMS}, ball_off=[0] * (F + 1), capacity=0, device=dev)
        P, nP = merge_proposals(r.ctx, empty, sites, site_off, out, ones, self.a_init, capacity=M)
        ev["accepted"] = nP
        if nP == 0:
            return
        if self._ys is None or self._ys.shape != yw.shape:
            self._zero = torch.zeros_like(yw)
            self._ys = torch.empty_like(yw)
        api.simulate_signals(r.ctx, r.A, P.balls, model, ball_off=P.ball_off, y=self._ys, B_cap=P.B_cap)
        Ls = api.residual_loss(r.ctx, self._ys, self._zero).cpu().numpy()
        T1, _ = merge_proposals(r.ctx, st, sites, site_off, out, ones, self.a_init, capacity=st.count() + nP)
        L1 = self._frame_losses(r, model, T1, y_k, yw)
        es = 0.5 * (L1 - L0 - Ls)
        alpha = np.where((Ls > 0.0) & (es < 0.0), np.minimum(-es / np.where(Ls > 0, Ls, 1.0), self.max_scale),
                         0.0).astype(np.float32)
        for _ in range(2):           # the judge: frames whose loss did not fall get no proposals
            if not np.any(alpha > 0):
                return
            try:
                new, _ = merge_proposals(r.ctx, st, sites, site_off, out, torch.as_tensor(alpha, device=dev),
                                         self.a_init, capacity=r.cap)
            except _abi.SbpError as e:
                if e.code != _abi.SBP_E_CAPACITY:
                    raise
                return
            L2 = self._frame_losses(r, model, new, y_k, yw)
            bad = (alpha > 0) & ~(L2 < L0) if self.judge else np.zeros(F, bool)
            if not np.any(bad):
                break
            alpha[bad] = 0.0
        else:
            return
        r.state = new
        ev.update(scale=float(alpha.max()), loss_after=float(L2.sum()), frames_kept=int((alpha > 0).sum()))
        ev["kept"] = True

    def _propose(self, r, model, y_k, yw, ev):
        st = r.state
        if st.F != 1:
            return self._propose_frames(r, model, y_k, yw, ev)
        L0 = _residual(r, model, y_k, yw)
        ev.update(loss_before=L0, loss_after=L0)
        M, X, sites = self.builder.build(r.A, st, model, yw)
        ev["candidates"] = M
        if M == 0:
            return
        out = self.mlp.forward(X)
        n_old = st.count()
        try:
            n_new = append_proposals(r.ctx, st, sites, out, M, self.a_init)
        except _abi.SbpError as e:
            if e.code != _abi.SBP_E_CAPACITY:
                raise
            return
        ev["accepted"] = n_new - n_old
        if n_new == n_old:
            return
        dev = yw.device
        if self._zero is None or self._zero.shape != yw.shape:
            self._zero = torch.zeros_like(yw)
            self._ys = torch.empty_like(yw)
            self._off = torch.zeros(2, dtype=torch.int64, device=dev)
        self._off[0], self._off[1] = n_old, n_new
        api.simulate_signals(r.ctx, r.A, st.balls, model, ball_off=self._off, y=self._ys, B_cap=st.B_cap)
        Ls = float(api.residual_loss(r.ctx, self._ys, self._zero).sum().item())
        L1 = _residual(r, model, y_k, yw)
        st.ball_off[1:2].fill_(n_old)
        es = 0.5 * (L1 - L0 - Ls)
        if not (Ls > 0.0 and es < 0.0):
            return
        alpha = min(-es / Ls, self.max_scale)
        append_proposals(r.ctx, st, sites, out, M, self.a_init, p0_scale=alpha)
        L2 = _residual(r, model, y_k, yw)
        ev.update(scale=alpha, loss_after=L2)
        if self.judge and not L2 < L0:
            st.ball_off[1:2].fill_(n_old)
        else:
            ev["kept"] = True


# ---------------------------------------------------------- data & A/B --

def proposal_workload(index, n_init=200_000, n_det=512):
    """A conformal-array workload (the 512-element jittered ellipsoid, a
    branching-tree phantom, 2048 samples at 40 MHz) from seed stream 5."""
    rng = synth.rng_for(5, index)
    arr = synth.ellipsoid_array(n_det, (20.0, 15.0, 10.0), rng, jitter=1.0)
    region = synth.Region(10.0, (18.0, 13.0, 8.0))
    gt = synth.drop_near(synth.tree_phantom(rng, region), arr, 1.5)
    init = synth.drop_near(synth.region_init(rng, region, n_init), arr, 1.5)
    return synth.Workload(f"proposal-{index}", arr, gt, init, 2048, 0.025, (4, 2, 1), 0.1)


def synthetic_measurement(ctx, wl, noise=0.05, seed=0, device="cuda:0", sampling=api.SAMPLING_BIN):
    dev = torch.device(device)
    A = {k: torch.as_tensor(v, device=dev) for k, v in wl.array.items()}
    gt = {k: torch.as_tensor(v, device=dev) for k, v in wl.gt.items()}
    y = api.simulate_signals(ctx, A, gt, api.Model(c=synth.C, dt=wl.dt, T=wl.T, f=1, sampling=sampling))
    if noise > 0:
        rng = np.random.default_rng(seed)
        sigma = noise * float(y.abs().max())
        y = y + sigma * torch.as_tensor(rng.normal(size=tuple(y.shape)).astype(np.float32), device=dev)
    return y.contiguous()


def default_schedule(levels, iters=60, grow_every=20):
    return recon.plain_schedule(levels, iters=iters, coarse_grow_every=grow_every,
                                fine_grow_every=grow_every, softplus_frac=0.2, tol=1e-3)


def label_events(events, grid: Grid, final_mass, threshold=0.1):
    """(X, grow label, p0 target) from recorded events and the final cell masses."""
    fm = np.asarray(final_mass, np.float64).reshape(grid.nx, grid.ny, grid.nz)
    Xs, ys, ps = [], [], []
    for ev in events:
        xyz = ev["xyz"]
        idx = np.rint((xyz - np.array([grid.ox, grid.oy, grid.oz])) / grid.h - 0.5).astype(np.int64)
        idx = np.clip(idx, 0, np.array([grid.nx, grid.ny, grid.nz]) - 1)
        m = fm[idx[:, 0], idx[:, 1], idx[:, 2]]
        Xs.append(ev["X"])
        ys.append((m > threshold).astype(np.float32))
        ps.append(np.where(m > threshold, m, 0.0).astype(np.float32))
    return np.concatenate(Xs), np.concatenate(ys), np.concatenate(ps)


def plain_run(ctx, wl, y, stages, builder=None, capacity=0, graph_iters=0, stop_below=None, proposer=None):
    cfg = recon.ReconConfig(stages=stages, T=wl.T, dt=wl.dt, dup_frac=0.05, capacity=capacity,
                            graph_iters=graph_iters)
    r = recon.Recon(wl.array, y, wl.init, cfg, ctx=ctx)
    r.proposer = proposer
    return r, r.run(stop_below=stop_below)


def generate(ctx, indices, grid: Grid, stages, workload=proposal_workload, log=print, labels="phantom",
             neg_frac=1.0, **wl_kw):
    """Training set from plain reconstructions of the given workload indices.

    labels = "phantom": a candidate is labelled by the seeded phantom's mass in
    its cell (the reconstructions are of synthetic phantoms, so the answer the
    network should give is known); "final": by the mass the plain
    reconstruction ends up with in the cell.  neg_frac < 1 keeps every positive
    site and a seeded random fraction of the negative ones (the balanced
    "auto" class weight of train() is unchanged by it)."""
    builder = FeatureBuilder(ctx, grid, a_probe=0.1, half=-grid.ox)
    Xs, ys, ps = [], [], []
    for i in indices:
        wl = workload(i, **wl_kw)
        y = synthetic_measurement(ctx, wl, seed=50_000 + i)
        rec = Recorder(builder)
        r, out = plain_run(ctx, wl, y, stages, proposer=rec, capacity=4 * len(wl.init["x"]))
        if labels == "phantom":
            gt = {k: torch.as_tensor(np.asarray(v, np.float32), device=r.dev) for k, v in wl.gt.items()}
            off = torch.tensor([0, len(wl.gt["x"])], dtype=torch.int64, device=r.dev)
            fm = grid_mass(ctx, gt, off, grid).cpu().numpy()
        elif labels == "final":
            st = out["state"]
            fm = grid_mass(ctx, st.balls, st.ball_off, grid, B_cap=st.B_cap).cpu().numpy()
        else:
            raise ValueError(f"unknown labels {labels!r}")
        if rec.events:
            X, yg, yp = label_events(rec.events, grid, fm)
            if neg_frac < 1.0:
                keep = (yg > 0.5) | (np.random.default_rng(70_000 + i).random(len(yg)) < neg_frac)
                X, yg, yp = X[keep], yg[keep], yp[keep]
            Xs.append(X), ys.append(yg), ps.append(yp)
        log(json.dumps(dict(event="plain-run", index=i, wall_s=round(out["wall_s"], 3),
                            final_loss=out["final_loss"], growth_points=len(rec.events),
                            samples=int(sum(len(e["X"]) for e in rec.events)),
                            positives=float(np.mean(ys[-1])) if rec.events else None)), flush=True)
    return np.concatenate(Xs), np.concatenate(ys), np.concatenate(ps)


def train(mlp: ProposalMLP, X, yg, yp, epochs=4, batch=8192, lr=1e-3, seed=0, log=print, pos_weight=1.0):
    """Minibatch Adam on the GPU; returns the per-epoch mean losses.  With
    pos_weight = 1 the classes are not re-weighted (a site is accepted where
    the network's P(grow) > 1/2); "auto" weighs the positives by the
    negatives-to-positives ratio of the training set."""
    rng = np.random.default_rng(seed)
    n = len(X)
    if pos_weight == "auto":
        p = float(np.mean(yg))
        pos_weight = (1.0 - p) / p if 0.0 < p < 1.0 else 1.0
    order = rng.permutation(n)
    dev = mlp.dev
    Xd = torch.as_tensor(np.ascontiguousarray(X[order], np.float32), device=dev)
    gd = torch.as_tensor(np.ascontiguousarray(yg[order], np.float32), device=dev)
    pd = torch.as_tensor(np.ascontiguousarray(yp[order], np.float32), device=dev)
    hist = []
    for ep in range(epochs):
        start = int(rng.integers(0, min(batch, n - batch + 1))) if n > batch else 0
        losses = []
        for s in range(start, n - batch + 1 if n >= batch else 1, batch):
            e = min(s + batch, n)
            losses.append(mlp.train_step(Xd[s:e], gd[s:e], pd[s:e], pos_weight=pos_weight, lr=lr))
        L = float(torch.stack(losses).mean().item())
        hist.append(L)
        log(json.dumps(dict(event="epoch", epoch=ep, loss=L, batches=len(losses), pos_weight=pos_weight)),
            flush=True)
    return hist


def auc(score, label):
    """Area under the ROC curve (ties count one half) of scores against 0/1 labels."""
    from scipy.stats import rankdata
    label = np.asarray(label) > 0.5
    npos, nneg = int(label.sum()), int((~label).sum())
    if npos == 0 or nneg == 0:
        return None
    r = rankdata(np.asarray(score, np.float64))
    return float((r[label].sum() - npos * (npos + 1) / 2.0) / (npos * nneg))


def first_below(log, target):
    """Time of the first final-stage iteration whose loss is <= target (None if none)."""
    last = max(e["stage"] for e in log)
    for e in log:
        if e["kind"] == "iter" and e["stage"] == last and e["loss"] <= target:
            return e["t"]
    return None


def compare(ctx, mlp, stages, grid, evals, n_init, when=(0,), max_per_stage=None, patience=1,
            reprobe_every=None, graph_iters=0, labels="final", first_index=10_000, log=print):
    """Wall time to the plain method's final residual with and without the
    network on `evals` held-out phantoms (seeds first_index + j), run one
    after the other with one proposer (so a gate that carries over runs,
    reprobe_every, sees them in order), and the network's held-out AUC on the
    candidate sites of the plain runs."""
    rows, scores, labs = [], [], []
    builder = FeatureBuilder(ctx, grid, a_probe=0.1, half=-grid.ox)
    lp = LearnedProposer(mlp, builder, stages=list(when) if when else None,
                         max_per_stage=max_per_stage, patience=patience, reprobe_every=reprobe_every)
    for j in range(evals):
        i = first_index + j
        wl = proposal_workload(i, n_init=n_init)
        y = synthetic_measurement(ctx, wl, seed=60_000 + j)
        cap = 4 * len(wl.init["x"])
        rec = Recorder(builder)
        _, plain = plain_run(ctx, wl, y, stages, capacity=cap, proposer=rec)
        # runs differ by FP32 summation order (~1e-5 relative): the target is
        # the plain final loss plus a 1e-3 relative margin, for every run
        target = plain["final_loss"] * (1.0 + 1e-3)
        _, plain2 = plain_run(ctx, wl, y, stages, capacity=cap, stop_below=target,
                              graph_iters=graph_iters)
        lp.a_init = wl.a_init
        lp.new_run()
        n_ev = len(lp.events)
        _, learned = plain_run(ctx, wl, y, stages, capacity=cap, stop_below=target, proposer=lp,
                               graph_iters=graph_iters)
        if rec.events:
            st = plain["state"]
            if labels == "phantom":
                gt = {k: torch.as_tensor(np.asarray(v, np.float32), device=mlp.dev) for k, v in wl.gt.items()}
                off = torch.tensor([0, len(wl.gt["x"])], dtype=torch.int64, device=mlp.dev)
                fm = grid_mass(ctx, gt, off, grid).cpu().numpy()
            else:
                fm = grid_mass(ctx, st.balls, st.ball_off, grid, B_cap=st.B_cap).cpu().numpy()
            X, yg, _ = label_events(rec.events, grid, fm)
            out = mlp.forward(torch.as_tensor(X, device=mlp.dev)).cpu().numpy()
            scores.append(out[:, 0])
            labs.append(yg)
        row = dict(event="compare", index=i,
                   plain_s=plain2["t_target"] or plain2["wall_s"], plain_reached=plain2["t_target"] is not None,
                   plain_final_loss=plain["final_loss"],
                   learned_s=learned["t_target"] or learned["wall_s"],
                   learned_reached=learned["t_target"] is not None, learned_final_loss=learned["final_loss"],
                   proposals_tried=len(lp.events) - n_ev,
                   proposals_kept=sum(e["kept"] for e in lp.events[n_ev:]),
                   gate_closed=lp.gated, proposal_s=sum(e.get("seconds", 0.0) for e in lp.events[n_ev:]))
        rows.append(row)
        log(json.dumps(row), flush=True)
    S = np.concatenate(scores) if scores else np.zeros(0)
    Lb = np.concatenate(labs) if labs else np.zeros(0)
    plain_s = float(np.sum([r["plain_s"] for r in rows]))
    learned_s = float(np.sum([r["learned_s"] for r in rows]))
    return dict(rows=rows, phantoms=evals, plain_s=plain_s, learned_s=learned_s,
                speedup=plain_s / learned_s if learned_s > 0 else None,
                per_phantom_speedup=[r["plain_s"] / r["learned_s"] for r in rows],
                reached=sum(r["learned_reached"] for r in rows),
                heldout_auc=auc(S, Lb), heldout_sites=int(len(Lb)),
                heldout_positives=float(np.mean(Lb)) if len(Lb) else None)


def frames_workload(index=0, n_frames=16, lo=100_000, hi=2_000_000):
    """The batched workload: frames of the conformal workload's array whose
    phantom is shifted within 1 mm and rescaled per frame, with per-frame
    initial clouds log-uniform in [lo, hi] balls."""
    base = synth.conformal_config(seed_index=index)
    gts, inits = synth.batched_frames(base, n_frames, seed_index=index, lo=lo, hi=hi)
    return base, gts, inits


def frames_measurement(ctx, base, gts, noise=0.05, seed=0, device="cuda:0"):
    dev = torch.device(device)
    A = {k: torch.as_tensor(v, device=dev) for k, v in base.array.items()}
    model = api.Model(c=synth.C, dt=base.dt, T=base.T, f=1)
    ys = [api.simulate_signals(ctx, A, {k: torch.as_tensor(v, device=dev) for k, v in g.items()}, model)[0]
          for g in gts]
    y = torch.stack(ys)
    if noise > 0:
        rng = np.random.default_rng(seed)
        sigma = noise * float(y.abs().max())
        y = y + sigma * torch.as_tensor(rng.normal(size=tuple(y.shape)).astype(np.float32), device=dev)
    return y.contiguous()


def frames_run(ctx, base, y, inits, stages, proposer=None, stop_below=None, graph_iters=0):
    balls = synth.concat_balls(inits)
    off = np.cumsum([0] + [len(b["x"]) for b in inits]).tolist()
    cfg = recon.ReconConfig(stages=stages, T=base.T, dt=base.dt, dup_frac=0.05, capacity=2 * off[-1],
                            graph_iters=graph_iters)
    r = recon.Recon(base.array, y, balls, cfg, ball_off=off, ctx=ctx)
    r.proposer = proposer
    return r, r.run(stop_below=stop_below)


def compare_frames(ctx, mlp, stages, grid, n_frames=16, lo=100_000, hi=2_000_000, index=0, when=(0,),
                   patience=1, graph_iters=0, log=print):
    """Learned + batched against plain batched: wall time of one batched
    reconstruction (all frames in every call) to the plain run's final loss
    summed over the frames."""
    base, gts, inits = frames_workload(index, n_frames, lo, hi)
    y = frames_measurement(ctx, base, gts, seed=80_000 + index)
    _, plain = frames_run(ctx, base, y, inits, stages, graph_iters=graph_iters)
    target = plain["final_loss"] * (1.0 + 1e-3)
    _, plain2 = frames_run(ctx, base, y, inits, stages, stop_below=target, graph_iters=graph_iters)
    lp = LearnedProposer(mlp, FeatureBuilder(ctx, grid, a_probe=0.1, half=-grid.ox), a_init=base.a_init,
                         stages=list(when) if when else None, patience=patience)
    lp.new_run()
    _, learned = frames_run(ctx, base, y, inits, stages, proposer=lp, stop_below=target, graph_iters=graph_iters)
    row = dict(event="compare-frames", frames=n_frames, balls=int(sum(len(b["x"]) for b in inits)),
               plain_s=plain2["t_target"] or plain2["wall_s"], plain_reached=plain2["t_target"] is not None,
               plain_final_loss=plain["final_loss"], learned_s=learned["t_target"] or learned["wall_s"],
               learned_reached=learned["t_target"] is not None, learned_final_loss=learned["final_loss"],
               proposals_tried=len(lp.events), proposals_kept=sum(e["kept"] for e in lp.events),
               frames_kept=[e.get("frames_kept", 0) for e in lp.events], gate_closed=lp.gated,
               proposal_s=sum(e.get("seconds", 0.0) for e in lp.events))
    row["speedup"] = row["plain_s"] / row["learned_s"]
    log(json.dumps(row), flush=True)
    return row


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the growth-proposal network on plain runs and "
                                             "compare wall time to the plain final residual.")
    ap.add_argument("--train", type=int, default=16, help="plain reconstructions for training")
    ap.add_argument("--eval", type=int, default=4, help="held-out phantoms for the comparison")
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--n-init", type=int, default=200_000)
    ap.add_argument("--train-n-init", type=int, default=None,
                    help="initial cloud of the training runs (default: --n-init)")
    ap.add_argument("--labels", choices=("phantom", "final"), default="final")
    ap.add_argument("--pos-weight", default="auto", help="a number, or auto (negatives / positives)")
    ap.add_argument("--patience", type=int, default=1,
                    help="rejected proposals in a row after which the network stays off (0: never)")
    ap.add_argument("--reprobe-every", type=int, default=0,
                    help="carry the gate over the runs, reopening it for one probe every N runs "
                         "(0: the gate is per run)")
    ap.add_argument("--neg-frac", type=float, default=1.0,
                    help="fraction of the negative training sites kept (all positives are)")
    ap.add_argument("--when", default="0", help="comma-separated stage indices the network acts in "
                                                "(default: the coarse stage, where its proposals are kept)")
    ap.add_argument("--max-per-stage", type=int, default=None)
    ap.add_argument("--graph-iters", type=int, default=0,
                    help="iterations per captured HIP graph in the timed runs")
    ap.add_argument("--frames", type=int, default=0,
                    help="compare learned + batched against plain batched on this many frames of the "
                         "batched workload instead (with --load-weights)")
    ap.add_argument("--frame-balls", default="100000,2000000",
                    help="lo,hi of the per-frame initial cloud (log-uniform) for --frames")
    ap.add_argument("--load-weights", default=None, help="skip training: use these weights")
    ap.add_argument("--save-weights", default=None, help="write the trained weights (BF16) here")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    ctx = api.context(0)
    grid = Grid.cube(10.0, 0.2)
    stages = default_schedule((4, 2, 1), iters=args.iters)
    pw = args.pos_weight if args.pos_weight == "auto" else float(args.pos_weight)
    t_gen = t_train = 0.0
    hist, n_samples, positives = [], 0, None
    if args.load_weights:
        mlp = ProposalMLP.load(ctx, args.load_weights)
    else:
        t0 = time.perf_counter()
        X, yg, yp = generate(ctx, range(args.train), grid, stages, labels=args.labels,
                             n_init=args.train_n_init or args.n_init, neg_frac=args.neg_frac)
        t_gen = time.perf_counter() - t0
        n_samples, positives = len(X), float(np.mean(yg))
        mlp = ProposalMLP(ctx, seed=0)
        t0 = time.perf_counter()
        hist = train(mlp, X, yg, yp, epochs=args.epochs, pos_weight=pw)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del X, yg, yp
        if args.save_weights:
            mlp.save(args.save_weights, bf16=True)
    when = [int(v) for v in args.when.split(",") if v != ""] or None
    if args.frames > 0:
        lo, hi = (int(v) for v in args.frame_balls.split(","))
        rows = [compare_frames(ctx, mlp, stages, grid, args.frames, lo, hi, index=j, when=when,
                               patience=args.patience or None, graph_iters=args.graph_iters)
                for j in range(max(args.eval, 1))]
        if args.out:
            with open(args.out, "w") as fh:
                json.dump(dict(rows=rows), fh, indent=1)
        return 0
    res = compare(ctx, mlp, stages, grid, args.eval, args.n_init, when=when,
                  max_per_stage=args.max_per_stage, patience=args.patience or None,
                  reprobe_every=args.reprobe_every or None, graph_iters=args.graph_iters,
                  labels=args.labels)
    summary = dict(event="summary", train_runs=0 if args.load_weights else args.train,
                   labels=args.labels, pos_weight=pw, neg_frac=args.neg_frac, patience=args.patience,
                   reprobe_every=args.reprobe_every, samples=n_samples, positives=positives,
                   generate_s=t_gen, train_s=t_train, epoch_losses=hist,
                   **{k: v for k, v in res.items() if k != "rows"})
    print(json.dumps(summary), flush=True)
    if args.save_weights and not args.load_weights:
        meta = {k: summary[k] for k in ("train_runs", "labels", "pos_weight", "neg_frac", "samples",
                                        "positives", "epoch_losses", "heldout_auc", "heldout_sites")}
        meta.update(n_init=args.train_n_init or args.n_init, epochs=args.epochs, iters=args.iters,
                    command="python -m paper_2601_00551_amd.proposal " + " ".join(argv or sys.argv[1:]))
        with open(args.save_weights[:-4] + ".json", "w") as fh:
            json.dump(meta, fh, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(dict(rows=res["rows"], summary=summary), fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
