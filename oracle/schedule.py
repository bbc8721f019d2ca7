"""Algorithm 1 (the coarse-to-fine schedule) as a plain FP64 composition of the
oracle's steps.  TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The paper gives the schedule's structure (Algorithm 1; sections 4.1-4.3) but
not its constants; this module takes the same readings as the library's host
driver, written out step by step:

for each sampling rate f_k, lowest first (one stage per rate):
  1. y^(k) = Downsample_{f_k}(y_real)                           (section 4.3)
  2. zero-gradient filtering of the cloud at that rate          (section 4.2)
  3. at a fine stage, one point duplication with the gradients of the
     current cloud (the growth rule with dup_frac)               (section 4.3)
  4. Adam moments start at zero, step count 1
  5. ``iters`` iterations of: simulate, L = ||y_sim - y^(k)||^2, back-
     propagation, Adam on the stage's parameters (coarse: p0 and a; fine: all
     five, section 4.1); after every ``grow_every`` iterations (not after the
     last, not during the refinement) split / destroy with the gradients of
     the last iteration -- the position gradients of a coarse stage are never
     computed there and stay zero, so a split there is along x
  6. the last ``softplus_frac`` of the iterations of the stage optimise a~
     with a = softplus(a~) (section 4.3): at the switch a~ = softplus^-1(a)
     and the moments of a restart at zero; at the stage end a = softplus(a~).

Every step that changes the cloud returns fresh (zero) gradient arrays, as
the library's state does after filtering and growth.  One frame.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import (PARAMS, GrowthRule, Time, adam_step, downsample, filter_zero_grad, grow,
               residual_loss, sigmoid, simulate, softplus, softplus_inv, vjp)

COARSE = ("p0", "a")
ALL = PARAMS


@dataclasses.dataclass
class Stage:
    f: int
    mask: tuple = ALL
    iters: int = 5
    filter: bool = True
    duplicate: bool = False
    grow_every: int = 0
    softplus_frac: float = 0.0


@dataclasses.dataclass
class Config:
    base: Time                               # the measured record's time grid (f = 1)
    stages: list
    lr: tuple = (0.005, 0.005, 0.005, 0.02, 0.002)   # x, y, z, p0, a
    growth: dict = dataclasses.field(default_factory=lambda: dict(
        destroy_frac=0.02, a_min=0.02, a_split=0.3, dup_offset=0.5))
    dup_frac: float = 0.1


@dataclasses.dataclass
class State:
    balls: dict                              # FP64 arrays; "a" holds a~ while softplus is on
    grad: dict
    m: dict
    v: dict
    softplus: bool = False

    @staticmethod
    def start(balls):
        n = len(np.asarray(balls["x"]))
        z = {k: np.zeros(n) for k in PARAMS}
        return State({k: np.asarray(balls[k], dtype=np.float64).copy() for k in PARAMS},
                     dict(z), {k: np.zeros(n) for k in PARAMS}, {k: np.zeros(n) for k in PARAMS})

    def count(self):
        return len(self.balls["x"])


def level(base: Time, f: int) -> Time:
    """The time grid of the level with downsampling factor f (section 4.3)."""
    return Time(c=base.c, dt=base.dt, t0=base.t0, T=base.T // f, f=f, profile=base.profile,
                directivity=base.directivity, K=base.K, sampling=base.sampling)


def sizes(st: State) -> dict:
    """The balls with the size the forward model sees (a = softplus(a~) when on)."""
    b = dict(st.balls)
    if st.softplus:
        b["a"] = softplus(st.balls["a"])
    return b


def loss_and_gradients(st: State, arr, tm: Time, y_k):
    """L and dL/dtheta for all five parameters (dL/da~ = dL/da sigmoid(a~))."""
    b = sizes(st)
    L, v = residual_loss(simulate(b, arr, tm), y_k)
    g = vjp(b, arr, tm, v)
    if st.softplus:
        g["a"] = g["a"] * sigmoid(st.balls["a"])
    return L, g


def filter_step(st: State, arr, tm: Time, y_k):
    """Zero-gradient filtering; the kept balls keep their moments."""
    keep, g, out = filter_zero_grad(st.balls, arr, tm, y_k, strict=True)
    n = int(keep.sum())
    new = State({k: np.asarray(out[k], dtype=np.float64) for k in PARAMS}, {k: np.zeros(n) for k in PARAMS},
                {k: st.m[k][keep] for k in PARAMS}, {k: st.v[k][keep] for k in PARAMS}, st.softplus)
    return new, keep, g


def grow_step(st: State, rule: GrowthRule):
    """The growth rule with the state's gradients; new balls get zero moments."""
    out, _, born, src = grow(st.balls, st.grad, rule)
    n = len(src)
    m = {k: np.where(born, 0.0, st.m[k][src]) for k in PARAMS}
    v = {k: np.where(born, 0.0, st.v[k][src]) for k in PARAMS}
    return State(out, {k: np.zeros(n) for k in PARAMS}, m, v, st.softplus), born, src


def iteration(st: State, arr, tm: Time, y_k, mask, lr, step: int):
    """One iteration; returns the loss before the update.  Gradients outside the
    mask are left as they were (the library does not compute them)."""
    L, g = loss_and_gradients(st, arr, tm, y_k)
    for i, k in enumerate(PARAMS):
        if k not in mask:
            continue
        st.grad[k] = g[k]
        st.balls[k], st.m[k], st.v[k] = adam_step(st.balls[k], g[k], st.m[k], st.v[k], step, lr[i])
    return L


def softplus_switch(st: State, on: bool):
    """a -> a~ = softplus^-1(a) (on) or a~ -> a = softplus(a~) (off); the
    moments of the size restart at zero."""
    st.balls["a"] = softplus_inv(st.balls["a"]) if on else softplus(st.balls["a"])
    st.m["a"] = np.zeros_like(st.m["a"])
    st.v["a"] = np.zeros_like(st.v["a"])
    st.softplus = on


def rule(cfg: Config, dup_frac: float) -> GrowthRule:
    return GrowthRule(dup_frac=dup_frac, **cfg.growth)


def run(init, arr, y_real, cfg: Config):
    """The whole schedule.  Returns (final state, per-stage records): each record
    holds the ball counts after filtering and after duplication and the loss of
    every iteration."""
    st = State.start(init)
    records = []
    for stg in cfg.stages:
        tm = level(cfg.base, stg.f)
        y_k = downsample(y_real, stg.f)
        rec = {"f": stg.f, "count_in": st.count()}
        if stg.filter:
            st, _, _ = filter_step(st, arr, tm, y_k)
        rec["count_filtered"] = st.count()
        if stg.duplicate and cfg.dup_frac > 0:
            _, st.grad = loss_and_gradients(st, arr, tm, y_k)
            st, _, _ = grow_step(st, rule(cfg, cfg.dup_frac))
        rec["count_entry"] = st.count()
        st.m = {k: np.zeros(st.count()) for k in PARAMS}
        st.v = {k: np.zeros(st.count()) for k in PARAMS}
        step = 1
        sp_start = stg.iters - int(round(stg.softplus_frac * stg.iters)) if stg.softplus_frac > 0 else None
        losses = []
        it = 0
        while it < stg.iters:
            if sp_start is not None and it >= sp_start and not st.softplus:
                softplus_switch(st, True)
            losses.append(iteration(st, arr, tm, y_k, stg.mask, cfg.lr, step))
            step += 1
            it += 1
            if stg.grow_every and it % stg.grow_every == 0 and it < stg.iters and not st.softplus:
                st, _, _ = grow_step(st, rule(cfg, 0.0))
        if st.softplus:
            softplus_switch(st, False)
        rec["losses"] = losses
        rec["count_out"] = st.count()
        records.append(rec)
    return st, records
