"""Hierarchical coarse-to-fine reconstruction driver (host side).

Follows Algorithm 1 of SlingBAG Pro and sections 4.1-4.3: for each sampling
rate, lowest first,

  1. Downsample_{f_k} of the measured signal                  (section 4.3)
  2. zero-gradient filtering of the cloud at that rate          (section 4.2)
  3. fine stages only: point duplication at the change of rate  (section 4.3)
  4. iterations "until converged": simulate, L2 loss, backpropagate, Adam;
     the coarse stage updates p0 and a only, fine stages all five parameters;
     split / destroy every `grow_every` iterations              (section 4.1)
  5. the last fraction of the final stage optimises a~ with a = softplus(a~)
     (positivity-constrained refinement, section 4.3).

Every step runs in libsbp.so through the C-ABI; this module only sequences the
calls, decides convergence from the (host-copied) loss, logs, and writes /
reads checkpoints.  The stage structure, convergence rule, learning rates and
per-stage Adam restart are readings of what the paper leaves open, not values
it prints.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np
import torch

from . import api, autotune
from .api import ALL, COARSE, PARAMS


@dataclasses.dataclass
class Stage:
    f: int                      # downsampling factor of this level
    mask: int = ALL             # parameters updated (COARSE in the coarse stage)
    iters: int = 100            # iteration cap
    filter: bool = True         # zero-gradient filter at stage entry
    duplicate: bool = False     # duplicate points at stage entry (fine stages)
    grow_every: int = 0         # split / destroy every N iterations (0: never)
    tol: float = 1e-3           # stop when the loss fell by less than tol (relative) ...
    window: int = 10            # ... over the last `window` iterations
    softplus_frac: float = 0.0  # final fraction of the stage run on a~ (a = softplus(a~))


@dataclasses.dataclass
class ReconConfig:
    stages: list
    T: int                      # samples of the measured record (base rate)
    dt: float                   # base sample interval, us
    c: float = 1.5
    t0: float = 0.0
    profile: int = api.PROFILE_GAUSS
    directivity: int = api.DIR_COS
    gauss_K: float = 5.0
    sampling: int = api.SAMPLING_BIN   # POINT: point samples, pyramid by decimation
    tuning: str | None = autotune.DEFAULT_PATH   # launch-shape cache applied at stage entry (None: keep)
    lr: tuple = (0.005, 0.005, 0.005, 0.02, 0.002)   # x, y, z, p0, a
    growth: dict = dataclasses.field(default_factory=lambda: dict(
        destroy_frac=0.02, a_min=0.02, a_split=0.3, dup_offset=0.5))
    dup_frac: float = 0.1
    capacity: int = 0           # ball capacity per state (0: twice the initial count)
    graph_iters: int = 0        # > 0: capture this many iterations per HIP graph launch
    checkpoint_dir: str | None = None
    checkpoint_every: int = 0   # iterations between checkpoints (0: stage ends only)
    log_path: str | None = None

    def to_json(self):
        d = dataclasses.asdict(self)
        d["stages"] = [dataclasses.asdict(s) if not isinstance(s, dict) else s for s in self.stages]
        return json.dumps(d)


def plain_schedule(levels, iters=100, coarse_grow_every=20, fine_grow_every=20, softplus_frac=0.2,
                   filter_each_stage=True, tol=1e-3):
    """Algorithm 1's structure: the first (lowest) rate is the coarse stage, the
    following rates are fine stages that start with a duplication."""
    st = []
    for k, f in enumerate(levels):
        coarse = k == 0
        st.append(Stage(f=f, mask=COARSE if coarse else ALL, iters=iters,
                        filter=filter_each_stage or k == 0, duplicate=not coarse,
                        grow_every=coarse_grow_every if coarse else fine_grow_every, tol=tol,
                        softplus_frac=softplus_frac if k == len(levels) - 1 else 0.0))
    return st


class InjectedFailure(RuntimeError):
    """Raised by Recon.run(fail_at=...) to rehearse a crash between iterations."""


class Recon:
    """One (batched) reconstruction on one GPU."""

    def __init__(self, array, y_real, init, config: ReconConfig, ball_off=None, ctx=None,
                 device="cuda:0"):
        self.dev = torch.device(device)
        self.cfg = config
        self.ctx = ctx if ctx is not None else api.context(self.dev.index or 0)
        self.A = {k: torch.as_tensor(np.asarray(v), dtype=torch.float32, device=self.dev).contiguous()
                  for k, v in array.items()}
        y = torch.as_tensor(np.asarray(y_real) if not torch.is_tensor(y_real) else y_real,
                            dtype=torch.float32, device=self.dev)
        self.y_real = (y if y.dim() == 3 else y[None]).contiguous()
        self.F = self.y_real.shape[0]
        self.D = self.A["qx"].numel()
        n0 = int(len(np.asarray(init["x"])))
        self.cap = int(config.capacity or 2 * max(n0, 1))
        if ball_off is None:
            ball_off = [0, n0]
        self.state = api.State(init, ball_off=ball_off, capacity=self.cap, device=self.dev)
        self.log = []
        self.t_start = None
        self.last_loss = None
        # optional growth-point hook proposer(recon, stage_index, model, y_k, y_work),
        # called after each split / destroy / duplicate (the learned proposal)
        self.proposer = None
        self.softplus_on = False    # the size arrays hold a~ (a = softplus(a~)) right now

    # ------------------------------------------------------------ helpers --
    def model(self, f, a_softplus=0):
        c = self.cfg
        return api.Model(c=c.c, dt=c.dt, t0=c.t0, T=c.T // f, f=f, profile=c.profile,
                         directivity=c.directivity, gauss_K=c.gauss_K, a_softplus=a_softplus,
                         sampling=c.sampling)

    def _tune(self, model):
        """Install the cached launch shape for this level and the largest frame's
        current ball count (results do not depend on it beyond rounding)."""
        if self.cfg.tuning:
            n = int(torch.diff(self.state.ball_off).max().item()) if self.F else 0
            autotune.apply_cached(self.ctx, self.cfg.tuning, model, self.D, max(n, 1))

    def _rule(self, dup_frac):
        g = dict(self.cfg.growth)
        return api.GrowthRule(dup_frac=dup_frac, **g)

    def _filter(self, model, y_k):
        s = self.state
        out = api.State({k: np.zeros(0) for k in PARAMS}, ball_off=[0] * (s.F + 1),
                        capacity=self.cap, device=self.dev)
        api.filter_zero_grad(self.ctx, self.A, s.balls, model, y_k, ball_off=s.ball_off, strict=True,
                             out=out.balls, off_out=out.ball_off, B_cap=s.B_cap, moments=(s.m, s.v),
                             moments_out=(out.m, out.v))
        self.state = out

    def _gradients(self, model, y_k, y_work):
        s = self.state
        api.simulate_signals(self.ctx, self.A, s.balls, model, ball_off=s.ball_off, y=y_work, B_cap=s.B_cap)
        api.residual_loss(self.ctx, y_work, y_k, v_out=y_work)
        api.adjoint_gradients(self.ctx, self.A, s.balls, model, y_work, mask=ALL, ball_off=s.ball_off,
                              grad=s.grad, B_cap=s.B_cap)

    def _grow(self, dup_frac, si=None, model=None, y_k=None, y_work=None):
        new, _ = api.grow(self.ctx, self.state, self._rule(dup_frac), capacity=self.cap)
        self.state = new
        if self.proposer is not None and model is not None:
            self.proposer(self, si, model, y_k, y_work)

    def _reset_adam(self):
        for k in PARAMS:
            self.state.m[k].zero_()
            self.state.v[k].zero_()

    # -------------------------------------------------------- checkpoints --
    def _ckpt_path(self):
        return os.path.join(self.cfg.checkpoint_dir, "checkpoint.npz")

    def save_checkpoint(self, stage, it, step, softplus_on):
        if not self.cfg.checkpoint_dir:
            return
        os.makedirs(self.cfg.checkpoint_dir, exist_ok=True)
        n = self.state.count()
        arrays = {}
        for k in PARAMS:
            arrays["b_" + k] = self.state.balls[k][:n].cpu().numpy()
            arrays["m_" + k] = self.state.m[k][:n].cpu().numpy()
            arrays["v_" + k] = self.state.v[k][:n].cpu().numpy()
        arrays["ball_off"] = self.state.ball_off.cpu().numpy()
        meta = dict(stage=stage, it=it, step=step, softplus_on=bool(softplus_on), log=self.log,
                    config=json.loads(self.cfg.to_json()))
        tmp = self._ckpt_path() + ".tmp.npz"
        np.savez(tmp, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **arrays)
        os.replace(tmp, self._ckpt_path())

    def load_checkpoint(self):
        with np.load(self._ckpt_path()) as z:
            meta = json.loads(bytes(z["meta"]).decode())
            balls = {k: z["b_" + k] for k in PARAMS}
            st = api.State(balls, ball_off=z["ball_off"], capacity=self.cap, device=self.dev)
            n = len(balls["x"])
            for k in PARAMS:
                st.m[k][:n] = torch.as_tensor(z["m_" + k], device=self.dev)
                st.v[k][:n] = torch.as_tensor(z["v_" + k], device=self.dev)
        self.state = st
        self.log = meta["log"]
        return meta

    # --------------------------------------------------------------- run --
    def run(self, resume=False, fail_at=None, on_iter=None, stop_below=None):
        """Run the schedule.  stop_below: end as soon as the last stage's loss
        is at or below this value (the time is reported as t_target)."""
        cfg = self.cfg
        t_target = None
        start_stage, start_it, step, softplus_on = 0, 0, 1, False
        if resume:
            meta = self.load_checkpoint()
            start_stage, start_it, step, softplus_on = meta["stage"], meta["it"], meta["step"], meta["softplus_on"]
            self.softplus_on = softplus_on
        self.t_start = time.perf_counter()
        y_work = torch.empty(self.F, self.D, cfg.T, device=self.dev)
        loss = torch.zeros(self.F, dtype=torch.float64, device=self.dev)
        for si in range(start_stage, len(cfg.stages)):
            stg = cfg.stages[si]
            stg = Stage(**stg) if isinstance(stg, dict) else stg
            model = self.model(stg.f, a_softplus=int(softplus_on))
            T_k = model.T
            pyramid = api.decimate if cfg.sampling == api.SAMPLING_POINT else api.downsample
            y_k = pyramid(self.ctx, self.y_real, stg.f)
            yw = y_work.view(-1)[: self.F * self.D * T_k].view(self.F, self.D, T_k)
            fresh = not (resume and si == start_stage and start_it > 0)
            if fresh:
                self._tune(model)
                if stg.filter:
                    self._filter(model, y_k)
                if stg.duplicate and cfg.dup_frac > 0:
                    self._gradients(model, y_k, yw)
                    self._grow(cfg.dup_frac, si, model, y_k, yw)
                self._reset_adam()
                step, it0 = 1, 0
                self._log(si, -1, stg, None, "stage-entry")
            else:
                it0 = start_it
            self._tune(model)     # for the cloud the stage iterates on
            sp_start = stg.iters - int(round(stg.softplus_frac * stg.iters)) if stg.softplus_frac > 0 else None
            hist = []
            it = it0
            graph = None
            while it < stg.iters:
                if sp_start is not None and it >= sp_start and not softplus_on:
                    api.softplus_reparam(self.ctx, self.state, True)
                    softplus_on = self.softplus_on = True
                    model = self.model(stg.f, a_softplus=1)
                    graph = None
                # iterations until the next growth, refinement switch or stage end
                limit = stg.iters
                if stg.grow_every:
                    limit = min(limit, (it // stg.grow_every + 1) * stg.grow_every)
                if sp_start is not None and it < sp_start:
                    limit = min(limit, sp_start)
                if cfg.checkpoint_every:
                    limit = min(limit, (it // cfg.checkpoint_every + 1) * cfg.checkpoint_every)
                gi = cfg.graph_iters
                if gi > 0 and limit - it >= gi:
                    if graph is None:
                        graph = api.StepGraph(self.ctx, self.A, self.state, model, y_k, yw,
                                              api.AdamParams(lr=cfg.lr, step=step, mask=stg.mask),
                                              iters=gi, step0=step)
                    graph.step_dev.fill_(step)
                    graph.launch(stream=torch.cuda.current_stream(self.dev))
                    Ls = graph.loss.view(gi, self.F).sum(dim=1).cpu().numpy()
                else:
                    prm = api.AdamParams(lr=cfg.lr, step=step, mask=stg.mask)
                    api.step(self.ctx, self.A, self.state, model, y_k, yw, prm, loss=loss)
                    Ls = [float(loss.sum().item())]
                for L in Ls:
                    L = float(L)
                    hist.append(L)
                    self.last_loss = L
                    self._log(si, it, stg, L, "iter")
                    if on_iter:
                        on_iter(self, si, it, L)
                    step += 1
                    it += 1
                    if (stop_below is not None and t_target is None and si == len(cfg.stages) - 1
                            and L <= stop_below):
                        t_target = time.perf_counter() - self.t_start
                if t_target is not None:
                    break
                # no growth in the softplus refinement: the arrays hold a~ there
                if stg.grow_every and it % stg.grow_every == 0 and it < stg.iters and not softplus_on:
                    self._grow(0.0, si, model, y_k, yw)
                    graph = None
                if cfg.checkpoint_every and it % cfg.checkpoint_every == 0:
                    self.save_checkpoint(si, it, step, softplus_on)
                if fail_at is not None and (si, it) == tuple(fail_at):
                    raise InjectedFailure(f"injected failure after stage {si} iteration {it}")
                if (sp_start is None or it < sp_start) and len(hist) > stg.window:
                    old = hist[-1 - stg.window]
                    if old > 0 and (old - hist[-1]) / old < stg.tol:
                        if sp_start is not None and not softplus_on:
                            it = max(it, sp_start)      # converged: go to the refinement phase
                        else:
                            break
            graph = None
            if softplus_on:
                api.softplus_reparam(self.ctx, self.state, False)
                softplus_on = self.softplus_on = False
            resume = False
            self.save_checkpoint(si + 1, 0, 1, False)
        torch.cuda.synchronize(self.dev)
        return {"state": self.state, "log": self.log, "final_loss": self.last_loss,
                "wall_s": time.perf_counter() - self.t_start, "t_target": t_target}

    def _log(self, si, it, stg, L, kind):
        rec = {"stage": si, "it": it, "f": stg.f, "kind": kind, "loss": L,
               "balls": self.state.count(), "t": time.perf_counter() - (self.t_start or time.perf_counter())}
        self.log.append(rec)
        if self.cfg.log_path:
            with open(self.cfg.log_path, "a") as fh:
                fh.write(json.dumps(rec) + "\n")
