"""SlingBAG Pro against a SlingBAG-style schedule on the same synthetic data.

Section 2 and Table 1 of SlingBAG Pro compare it with the original SlingBAG:
same initial cloud, same learning rates, but SlingBAG has no zero-gradient
filtering and iterates at the full sampling rate only, while Pro filters the
cloud and raises the sampling rate level by level.  This module runs both on
one workload and records, every few iterations, the image quality of the
voxelised cloud against the voxelised phantom (MSE / PSNR / SSIM, on the GPU);
the time spent measuring is excluded from the reported wall times.  Both
schedules also run on point samples (the pressure at the sample times, with
the decimation pyramid) next to the bin means of the default path.

    python -m paper_2601_00551_amd.ablation --variants pro,slingbag,pro_point,slingbag_point --out a.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api, image, proposal, recon, synth


def slingbag_schedule(iters=60, grow_every=20, softplus_frac=0.2, tol=1e-3):
    """Coarse then fine stage, both at the full rate and without filtering."""
    return [recon.Stage(f=1, mask=api.COARSE, iters=iters, filter=False, duplicate=False,
                        grow_every=grow_every, tol=tol),
            recon.Stage(f=1, mask=api.ALL, iters=iters, filter=False, duplicate=True,
                        grow_every=grow_every, tol=tol, softplus_frac=softplus_frac)]


def pro_schedule(levels=(4, 2, 1), iters=60, grow_every=20, tol=1e-3):
    return recon.plain_schedule(levels, iters=iters, coarse_grow_every=grow_every,
                                fine_grow_every=grow_every, softplus_frac=0.2, tol=tol)


class QualityProbe:
    """on_iter hook: every `every` iterations, voxelise the cloud and compare it
    with the phantom's volume; keeps (time without probing, stage, it, loss,
    MSE, PSNR, SSIM)."""

    def __init__(self, ctx, gt_vol, grid, model, every=10):
        self.ctx, self.gt_vol, self.grid, self.model, self.every = ctx, gt_vol, grid, model, every
        self.scale = float(gt_vol.max())
        self.work = torch.empty(10 * grid.ncell, dtype=torch.float32, device=gt_vol.device)
        self.vox = torch.empty_like(gt_vol)
        self.overhead = 0.0
        self.rows = []

    def measure(self, r, si, it, L):
        t0 = time.perf_counter()
        st = r.state
        m = api.Model(profile=self.model.profile, gauss_K=self.model.gauss_K, a_softplus=int(r.softplus_on))
        image.voxelize(self.ctx, st.balls, st.ball_off[:2].contiguous(), m, self.grid, B_cap=st.B_cap,
                       vox=self.vox)
        out = image.metrics(self.ctx, self.vox, self.gt_vol, (self.grid.nx, self.grid.ny, self.grid.nz),
                            self.scale, work=self.work).cpu().numpy()
        t_run = time.perf_counter() - r.t_start - self.overhead
        self.rows.append(dict(t=t_run, stage=si, it=it, loss=L, balls=st.count(), mse=float(out[0]),
                              psnr=float(out[1]), ssim=float(out[2])))
        self.overhead += time.perf_counter() - t0

    def __call__(self, r, si, it, L):
        if it % self.every == self.every - 1:
            self.measure(r, si, it, L)


def run(ctx, wl, y, stages, grid, gt_vol, every=10, capacity=0, sampling=api.SAMPLING_BIN):
    cfg = recon.ReconConfig(stages=stages, T=wl.T, dt=wl.dt, dup_frac=0.05, capacity=capacity,
                            sampling=sampling)
    r = recon.Recon(wl.array, y, wl.init, cfg, ctx=ctx)
    probe = QualityProbe(ctx, gt_vol, grid, api.Model(), every=every)
    out = r.run(on_iter=probe)
    probe.measure(r, len(stages) - 1, -1, out["final_loss"])
    return dict(wall_s=out["wall_s"] - probe.overhead, final_loss=out["final_loss"],
                balls=out["state"].count(), trace=probe.rows)


def time_to(trace, psnr):
    for row in trace:
        if row["psnr"] >= psnr:
            return row["t"]
    return None


# (name, schedule, sampling): the bin-average path of the paper, and the same
# two schedules on point samples with the decimation pyramid
VARIANTS = {
    "pro": (pro_schedule, api.SAMPLING_BIN),
    "slingbag": (slingbag_schedule, api.SAMPLING_BIN),
    "pro_point": (pro_schedule, api.SAMPLING_POINT),
    "slingbag_point": (slingbag_schedule, api.SAMPLING_POINT),
}


def main(argv=None):
    ap = argparse.ArgumentParser(description="SlingBAG Pro vs a SlingBAG-style schedule")
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--variants", default="pro,slingbag",
                    help="comma-separated subset of " + ",".join(VARIANTS))
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    names = [v for v in args.variants.split(",") if v]
    for v in names:
        if v not in VARIANTS:
            ap.error(f"unknown variant {v!r}")
    ctx = api.context(0)
    dev = torch.device("cuda:0")
    grid = proposal.Grid.cube(10.0, 0.2)
    # untimed warm-up: first launches of each kernel and launch shape
    wl = synth.conformal_config(seed_index=0)
    ys = proposal.synthetic_measurement(ctx, wl, seed=2000)
    off = torch.tensor([0, len(wl.gt["x"])], dtype=torch.int64, device=dev)
    gt_vol = image.voxelize(ctx, {k: torch.as_tensor(np.asarray(v), device=dev) for k, v in wl.gt.items()},
                            off, api.Model(), grid)
    for name in names:
        sched, smp = VARIANTS[name]
        run(ctx, wl, ys, sched(iters=3), grid, gt_vol, capacity=4 * len(wl.init["x"]), sampling=smp)
    rows = []
    for s in range(args.seeds):
        wl = synth.conformal_config(seed_index=s)
        # each sampling mode fits a record made the same way (same noise draw)
        ys = {smp: proposal.synthetic_measurement(ctx, wl, seed=2000 + s, sampling=smp)
              for smp in {VARIANTS[v][1] for v in names}}
        gt = {k: torch.as_tensor(np.asarray(v), device=dev) for k, v in wl.gt.items()}
        off = torch.tensor([0, len(wl.gt["x"])], dtype=torch.int64, device=dev)
        gt_vol = image.voxelize(ctx, gt, off, api.Model(), grid)
        cap = 4 * len(wl.init["x"])
        res = {}
        for name in names:
            sched, smp = VARIANTS[name]
            res[name] = run(ctx, wl, ys[smp], sched(iters=args.iters), grid, gt_vol, capacity=cap,
                            sampling=smp)
            last = res[name]["trace"][-1]
            print(json.dumps(dict(event="run", seed=s, schedule=name, wall_s=res[name]["wall_s"],
                                  final_loss=res[name]["final_loss"], balls=res[name]["balls"],
                                  psnr=last["psnr"], ssim=last["ssim"], mse=last["mse"])), flush=True)
        target = min(res[n]["trace"][-1]["psnr"] for n in names)
        row = dict(seed=s, psnr_target=target, **{n + "_t": time_to(res[n]["trace"], target) for n in names},
                   **res)
        rows.append(row)
        print(json.dumps(dict(event="compare", seed=s, psnr_target=target,
                              **{n + "_t": row[n + "_t"] for n in names})), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rows, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
