"""Throughput of the sliding-ball reconstruction hot path on one MI355X.

One step is one pass of every step of the hot path over the large workload
(1,024 transducers on a 45 mm hemispherical cap around a 30 mm cube holding
2,000,000 balls; 4,096 samples at 40 MHz; Gaussian balls, cosine directivity):

    downsample the measured signal to the level       (Downsample_f, section 4.3)
    zero-gradient filter of the cloud                 (section 4.2, Algorithm 1)
    simulate -> residual + loss -> adjoint -> Adam    (section 4.1 / 4.2)
    plain growth rule (split / destroy / duplicate)   (section 4.1)

value = (balls entering the step) x (transducers) / (seconds per step): every
(ball, transducer) pair is carried through the whole pass once per step.
Inputs are resident in HBM before the timed region; every kernel is timed with
HIP events on the stream it runs on.  Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# --- algorithmic work per (ball, transducer) pair, in FP32 lane-operation
# issue slots; a transcendental counts 2 (exp2, rcp and sqrt issue at half the
# FMA rate on gfx950, as `bench.py --rates` measures).  Counted from the
# method's arithmetic, not from the kernels' instruction streams. ------------
OPS_GEOMETRY = 22        # per pair: offset, rho (sqrt), 1/rho, e_hat, cosine, window, amplitude (18 + 2 transcendentals)
# forward, the bin-mean formula of section 4.2 / 4.3 (one bin per support bin,
# E + 1 per pair): u, u^2 / (2 a^2), exp, minus e_K, scale, bin difference,
# accumulate (6 + 1 transcendental)
OPS_FWD_BIN = 8
# forward as computed (edge form: one value per support edge, E per pair):
# exponent as a quadratic in the edge offset (2), exp2, scale, accumulate
OPS_FWD_EDGE = 6
# adjoint as computed: per support edge one staged read and the moment sums
# (w e, three sums, the exponential's two-multiply recurrence); per block of
# 16 edges an exact restart (two exp2) and folding the block's moments; per
# pair S0..S2 and the five gradients (with the cosine term)
OPS_ADJ_EDGE = 6
OPS_ADJ_BLOCK = 17
OPS_ADJ_PAIR = 25
# filter as computed (p0 only, nested sum): per edge one FMA and one multiply;
# per block two exp2 and the block's offsets; per pair the p0 gradient
OPS_FLT_EDGE = 2
OPS_FLT_BLOCK = 8
OPS_FLT_PAIR = 3
ADJ_BLOCK_EDGES = 16
OPS_FWD_EDGE_UNIFORM = 7  # per edge, UNIFORM profile: u, u^2, a^2 - u^2, clamp, scale, difference, accumulate
OPS_FWD_SAMPLE_POINT = 8  # per sample, point sampling: u, u^2 k, exp, u e, scale, accumulate
VALU_PEAK = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock = 3.93e13 lane-ops/s
# 64-bit LDS atomic adds, lane-operations per clock per CU, measured by
# `bench.py --rates` (profiles/issue_rates.md): the fastest pattern measured
# (four lanes on each residue modulo 16, random otherwise), pseudo-random
# addresses in a 4096-entry row, and the forward's own pattern (40 edges per
# lane as ten four-edge blocks from a rotated start)
LDS_U64_BEST = 9.27
LDS_U64_RANDOM = 6.21
LDS_U64_FORWARD_ROTATED = 7.50
LDS_PEAK = 256 * 2.4e9 * LDS_U64_BEST


def edges_per_pair(a_sup, cdt):
    """Expected support edges of a pair (strictly inside |u| < a_sup): the
    support spans 2 a_sup / (c dt) edge intervals."""
    return 2.0 * a_sup / cdt


def algorithmic_ops(E):
    """Lane-operation slots per pair of the three VALU-bound kernels for E
    expected support edges."""
    blocks = -(-E // ADJ_BLOCK_EDGES)
    return {"forward": OPS_GEOMETRY + (E + 1) * OPS_FWD_BIN,
            "forward_as_computed": OPS_GEOMETRY + E * OPS_FWD_EDGE,
            "adjoint": OPS_GEOMETRY + OPS_ADJ_PAIR + E * OPS_ADJ_EDGE + blocks * OPS_ADJ_BLOCK,
            "filter": OPS_GEOMETRY + OPS_FLT_PAIR + E * OPS_FLT_EDGE + blocks * OPS_FLT_BLOCK}


KERNEL_SOURCES = {"k_forward_gz": ("paper_2601_00551_amd/csrc/forward.hip", "paper_2601_00551_amd/csrc/sbp_internal.hpp"),
                  "k_adjoint": ("paper_2601_00551_amd/csrc/adjoint.hip", "paper_2601_00551_amd/csrc/sbp_internal.hpp")}
KERNEL_NAMES = {"forward": "k_forward_gz<1>", "adjoint": "k_adjoint<float, 1, 1, true, sbp::NoSrc>",
                "filter": "k_adjoint<float, 1, 1, false, sbp::NoSrc>"}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_large.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), flags=re.S)
    if not m:
        return None
    entry = json.loads(m.group(1)).get(KERNEL_NAMES[kernel])
    if not entry:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[KERNEL_NAMES[kernel].split("<")[0]]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != entry["source_hash"]:
        return None
    return entry["read_bytes"] + entry["write_bytes"]


def cpu_baseline(wl, model_kw, n_balls_sample, rng_seed=0):
    """The FP64 oracle on a bounded sample of the same workload: forward + VJP
    of n_balls_sample balls against every transducer at the full record."""
    import numpy as np
    import oracle
    from oracle import build as oracle_build
    # the oracle compiled for this host's CPU (-O3 -march=native), as timed
    oracle.use_library(oracle_build.build(native=True))
    rng = np.random.default_rng(rng_seed)
    idx = np.sort(rng.choice(len(wl.init["x"]), size=n_balls_sample, replace=False))
    balls = {k: v[idx] for k, v in wl.init.items()}
    tm = oracle.Time(c=model_kw["c"], dt=model_kw["dt"], T=model_kw["T"], f=1,
                     profile=oracle.GAUSS, directivity=oracle.COS)
    D = len(wl.array["qx"])
    t0 = time.perf_counter()
    y = oracle.simulate(balls, wl.array, tm)
    t1 = time.perf_counter()
    v = rng.normal(size=y.shape)
    oracle.vjp(balls, wl.array, tm, v)
    t2 = time.perf_counter()
    pairs = n_balls_sample * D
    cores = oracle.num_threads()
    # one thread on a sixteenth of the sample
    n1 = max(1, n_balls_sample // 16)
    b1 = {k: arr[:n1] for k, arr in balls.items()}
    prev = cores
    oracle.set_threads(1)
    try:
        t3 = time.perf_counter()
        oracle.simulate(b1, wl.array, tm)
        oracle.vjp(b1, wl.array, tm, v)
        t4 = time.perf_counter()
    finally:
        oracle.set_threads(prev)
    return {"value": pairs / (t2 - t0), "unit": "pairs/s", "cores": cores, "cpu_model": cpu_model_name(),
            "kind": "oracle", "build": "gcc -O3 -march=native -fopenmp",
            "sample": f"{n_balls_sample} of the {len(wl.init['x'])} balls x all {D} transducers, "
                      f"T={model_kw['T']}: oracle forward {t1 - t0:.2f} s + VJP {t2 - t1:.2f} s",
            "single_thread": {"value": n1 * D / (t4 - t3), "unit": "pairs/s",
                              "sample": f"{n1} balls x {D} transducers, forward + VJP {t4 - t3:.2f} s"}}


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


MLP_FLOP_FWD = 2 * (31 * 256 + 2 * 256 * 256 + 256 * 2)   # per candidate row
BF16_PEAK = 2.5e15


def mlp_rates(ctx, dev, M=262144, reps=20):
    """The proposal network's matrix-core rates: inference over M candidate rows
    and one training step (forward, loss, backward, Adam) on M rows."""
    import numpy as np
    import torch
    from paper_2601_00551_amd import proposal
    net = proposal.ProposalMLP(ctx, device=dev, seed=0)
    rng = np.random.default_rng(7)
    X = torch.as_tensor(rng.normal(size=(M, 31)).astype(np.float32), device=dev)
    yg = torch.as_tensor((rng.uniform(size=M) > 0.9).astype(np.float32), device=dev)
    yp = torch.as_tensor(rng.uniform(size=M).astype(np.float32), device=dev)
    out = torch.empty((M, 2), device=dev)
    for _ in range(3):
        net.forward(X, out=out)
        net.train_step(X, yg, yp)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        net.forward(X, out=out)
    e[1].record()
    for _ in range(reps):
        net.train_step(X, yg, yp)
    e[2].record()
    torch.cuda.synchronize()
    t_fwd = e[0].elapsed_time(e[1]) / reps * 1e-3
    t_train = e[1].elapsed_time(e[2]) / reps * 1e-3
    fwd = MLP_FLOP_FWD * M / t_fwd
    train = 3 * MLP_FLOP_FWD * M / t_train
    return {"rows": M, "forward_ms": t_fwd * 1e3, "forward_TFLOPs": fwd / 1e12,
            "forward_frac_bf16_peak": fwd / BF16_PEAK, "train_step_ms": t_train * 1e3,
            "train_TFLOPs": train / 1e12, "train_frac_bf16_peak": train / BF16_PEAK}


WEIGHTS = os.path.join(ROOT, "paper_2601_00551_amd", "proposal_weights.npz")


def learned_vs_plain(ctx, n_init=200_000, evals=20, patience=1, reprobe_every=10):
    """The second half of the metric: wall time to the plain method's final
    residual with and without the growth-proposal network, on `evals` held-out
    conformal-array phantoms with the configuration's 200 000-ball initial
    cloud, run one after the other.  The network is the committed one
    (trained offline on plain reconstructions, see its .json beside it); it
    acts in the coarse stage, and its gate closes after `patience` proposals
    in a row that the loss judge rejected, reopening for one probe every
    `reprobe_every` runs.  Times: eager runs to the first final-stage
    iteration at or below the plain run's final loss plus 0.1 %."""
    import numpy as np
    from paper_2601_00551_amd import proposal
    grid = proposal.Grid.cube(10.0, 0.2)
    stages = proposal.default_schedule((4, 2, 1), iters=60)
    if not os.path.exists(WEIGHTS):
        raise SystemExit(f"{WEIGHTS} is missing: train it with python -m paper_2601_00551_amd.proposal "
                         "--save-weights")
    net = proposal.ProposalMLP.load(ctx, WEIGHTS)
    meta_path = WEIGHTS[:-4] + ".json"
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    res = proposal.compare(ctx, net, stages, grid, evals, n_init, when=(0,), patience=patience,
                           reprobe_every=reprobe_every, labels=meta.get("labels", "final"),
                           log=lambda *a, **k: None)
    rows = res["rows"]
    return {"workload": f"conformal-ell512-tree-T2048-40MHz, {n_init} initial balls",
            "plain_s": res["plain_s"], "learned_s": res["learned_s"], "speedup": res["speedup"],
            "per_phantom_speedup_min": float(np.min(res["per_phantom_speedup"])),
            "per_phantom_speedup_max": float(np.max(res["per_phantom_speedup"])),
            "phantoms": evals, "reached": res["reached"],
            "proposals_tried": int(sum(r["proposals_tried"] for r in rows)),
            "proposals_kept": int(sum(r["proposals_kept"] for r in rows)),
            "gate": {"patience": patience, "reprobe_every": reprobe_every},
            "heldout_auc": res["heldout_auc"], "heldout_sites": res["heldout_sites"],
            "train_runs": meta.get("train_runs"), "train_samples": meta.get("samples"),
            "labels": meta.get("labels")}


def _timed(fn, reps):
    """Average milliseconds of fn() over reps calls, bracketed by events on the current stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def suite(args):
    """The other workloads, one JSON line each: per-iteration latency of the tiny
    workload (eager vs graph), per-level rates of the conformal workload, the
    16-frame batched iteration (graph-captured), and the large workload with
    uniform balls."""
    import numpy as np
    import torch
    from paper_2601_00551_amd import api, autotune, synth

    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    c = 1.5

    def measured(wl, noise=0.05, seed=0):
        A = {k: torch.as_tensor(v, device=dev) for k, v in wl.array.items()}
        gt = {k: torch.as_tensor(v, device=dev) for k, v in wl.gt.items()}
        y = api.simulate_signals(ctx, A, gt, api.Model(c=c, dt=wl.dt, T=wl.T, f=1))
        if noise > 0:
            rng = np.random.default_rng(seed)
            y = y + noise * float(y.abs().max()) * torch.as_tensor(
                rng.normal(size=tuple(y.shape)).astype(np.float32), device=dev)
        return A, y.contiguous()

    def fwd_adj(A, st, model, y_k, reps=5):
        yw = torch.empty_like(y_k)
        f = lambda: api.simulate_signals(ctx, A, st.balls, model, ball_off=st.ball_off, y=yw, B_cap=st.B_cap)
        b = lambda: api.adjoint_gradients(ctx, A, st.balls, model, y_k, mask=api.ALL, ball_off=st.ball_off,
                                          grad=st.grad, B_cap=st.B_cap)
        f(), b()
        return _timed(f, reps), _timed(b, reps)

    def iteration_rates(A, st, model, y_k, iters=10, reps=3):
        yw = torch.empty_like(y_k)
        prm = api.AdamParams(step=1)
        loss = torch.empty(st.F, dtype=torch.float64, device=dev)
        eager = lambda: api.step(ctx, A, st, model, y_k, yw, prm, loss=loss)
        eager()
        g = api.StepGraph(ctx, A, st, model, y_k, yw, prm, iters=iters, step0=1)
        cur = torch.cuda.current_stream(dev)
        launch = lambda: g.launch(stream=cur)
        launch()
        # the clock drifts under sustained load: alternate eager and graph
        # runs three times and average the last two pairs, once it has settled
        te, tg = [], []
        for _ in range(3):
            te.append(_timed(eager, iters * reps))
            tg.append(_timed(launch, reps) / iters)
        g.close()
        return 0.5 * (te[1] + te[2]), 0.5 * (tg[1] + tg[2])

    def filtered(A, init, model, y_k, off=None):
        n = len(init["x"])
        st = api.State(init, ball_off=off, capacity=n, device=dev)
        out = api.State({k: np.zeros(0) for k in api.PARAMS}, ball_off=[0] * (st.F + 1), capacity=n, device=dev)
        run = lambda: api.filter_zero_grad(ctx, A, st.balls, model, y_k, ball_off=st.ball_off, out=out.balls,
                                           off_out=out.ball_off, B_cap=n)
        run()
        return out, _timed(run, 3)

    # tiny: launch-latency bound; a captured launch holds the workload's whole
    # reconstruction (50 iterations)
    wl = synth.tiny_config()
    A, y = measured(wl, noise=0.0)
    model = api.Model(c=c, dt=wl.dt, T=wl.T, f=1)
    tuned = autotune.apply_cached(ctx, args.tuning, model, len(wl.array["qx"]), len(wl.init["x"]))
    st = api.State(wl.init, device=dev)
    te, tg = iteration_rates(A, st, model, y, iters=50, reps=4)
    print(json.dumps({"workload": wl.name, "balls": len(wl.init["x"]), "transducers": len(wl.array["qx"]),
                      "us_per_iteration_eager": te * 1e3, "us_per_iteration_graph": tg * 1e3,
                      "graph_speedup": te / tg, "tuning": tuned}), flush=True)
    if args.tiny:
        ctx.close()
        return

    # conformal: per level, filter then forward + adjoint on the kept balls
    wl = synth.conformal_config()
    A, y = measured(wl)
    D = len(wl.array["qx"])
    for f in wl.levels:
        model = api.Model(c=c, dt=wl.dt, T=wl.T // f, f=f)
        autotune.apply_cached(ctx, args.tuning, model, D, len(wl.init["x"]))
        y_k = api.downsample(ctx, y, f)
        st, t_filter = filtered(A, wl.init, model, y_k)
        kept = st.count()
        autotune.apply_cached(ctx, args.tuning, model, D, kept)     # shapes for the kept cloud
        tf, tb = fwd_adj(A, st, model, y_k)
        te, tg = iteration_rates(A, st, model, y_k, iters=10, reps=2)
        print(json.dumps({"workload": wl.name, "level_f": f, "samples": wl.T // f,
                          "balls_in": len(wl.init["x"]), "balls_kept": kept, "transducers": D,
                          "filter_ms": t_filter, "filter_pairs_per_s": len(wl.init["x"]) * D / (t_filter * 1e-3),
                          "forward_ms": tf, "adjoint_ms": tb,
                          "fwd_adj_pairs_per_s": kept * D / ((tf + tb) * 1e-3),
                          "iteration_ms_eager": te, "iteration_ms_graph": tg}), flush=True)

    # batched: 16 uneven frames in one graph-captured iteration at 40 MHz
    base = wl
    gts, inits = synth.batched_frames(base)
    F = len(inits)
    ys = []
    for g_ in gts:
        gt = {k: torch.as_tensor(v, device=dev) for k, v in g_.items()}
        ys.append(api.simulate_signals(ctx, A, gt, api.Model(c=c, dt=base.dt, T=base.T, f=1))[0])
    y = torch.stack(ys)
    rng = np.random.default_rng(4000)
    y += 0.05 * float(y.abs().max()) * torch.as_tensor(rng.normal(size=tuple(y.shape)).astype(np.float32),
                                                       device=dev)
    balls = synth.concat_balls(inits)
    off = np.cumsum([0] + [len(b["x"]) for b in inits]).tolist()
    model = api.Model(c=c, dt=base.dt, T=base.T, f=1)
    autotune.apply_cached(ctx, args.tuning, model, D, max(np.diff(off)))
    st, t_filter = filtered(A, balls, model, y.contiguous(), off=off)
    kept_off = st.ball_off.cpu().numpy()
    kept = int(kept_off[-1])
    autotune.apply_cached(ctx, args.tuning, model, D, int(np.max(np.diff(kept_off))))
    tf, tb = fwd_adj(A, st, model, y.contiguous())
    te, tg = iteration_rates(A, st, model, y.contiguous(), iters=5, reps=2)
    print(json.dumps({"workload": "batched-16-frames-ell512-T2048-40MHz", "frames": F,
                      "balls_in": off[-1], "balls_kept": kept,
                      "kept_per_frame_min": int(np.min(np.diff(kept_off))),
                      "kept_per_frame_max": int(np.max(np.diff(kept_off))), "transducers": D,
                      "filter_ms": t_filter, "forward_ms": tf, "adjoint_ms": tb,
                      "fwd_adj_pairs_per_s": kept * D / ((tf + tb) * 1e-3),
                      "iteration_ms_eager": te, "iteration_ms_graph": tg,
                      "iteration_pairs_per_s_graph": kept * D / (tg * 1e-3)}), flush=True)

    # large, uniform balls
    wl = synth.large_config()
    A = {k: torch.as_tensor(v, device=dev) for k, v in wl.array.items()}
    model = api.Model(c=c, dt=wl.dt, T=wl.T, f=1, profile=api.PROFILE_UNIFORM)
    autotune.apply_cached(ctx, args.tuning, model, len(wl.array["qx"]), len(wl.init["x"]))
    st = api.State(wl.init, device=dev)
    y = api.simulate_signals(ctx, A, st.balls, model)
    tf, tb = fwd_adj(A, st, model, y)
    B, D = len(wl.init["x"]), len(wl.array["qx"])
    E = edges_per_pair(0.15, c * wl.dt)
    ops_f = B * D * (OPS_GEOMETRY + (E + 1) * OPS_FWD_EDGE_UNIFORM)     # E + 1 bins
    print(json.dumps({"workload": wl.name.replace("uniform2M", "uniform2M-uniformballs"), "profile": "uniform",
                      "forward_ms": tf, "adjoint_ms": tb, "fwd_adj_pairs_per_s": B * D / ((tf + tb) * 1e-3),
                      "forward_frac_alu": ops_f / (tf * 1e-3) / VALU_PEAK}), flush=True)

    # large, GAUSS balls, point samples (the pressure at the sample times)
    model = api.Model(c=c, dt=wl.dt, T=wl.T, f=1, sampling=api.SAMPLING_POINT)
    autotune.apply_cached(ctx, args.tuning, model, D, B)
    st = api.State(wl.init, device=dev)
    y = api.simulate_signals(ctx, A, st.balls, model)
    tf, tb = fwd_adj(A, st, model, y)
    _, t_filter = filtered(A, wl.init, model, y)
    S = 2.0 * 5.0 * 0.15 / (c * wl.dt)          # samples strictly inside a 0.15 mm ball's support
    ops_f = B * D * (OPS_GEOMETRY + S * OPS_FWD_SAMPLE_POINT)
    print(json.dumps({"workload": wl.name + "-point", "profile": "gauss", "sampling": "point",
                      "forward_ms": tf, "adjoint_ms": tb, "filter_ms": t_filter,
                      "fwd_adj_pairs_per_s": B * D / ((tf + tb) * 1e-3),
                      "forward_frac_alu": ops_f / (tf * 1e-3) / VALU_PEAK}), flush=True)
    ctx.close()


def response_leg(ctx, wl, A, model, args, ms_plain):
    """The same step with each transducer's impulse response in the model
    (2.02 MHz, 54 % means with a seeded spread): the measured record is the
    convolved one, the filter and the adjoint correlate first.  Reports the
    step time and rate with the response on (the cloud then evolves
    differently, so its ball counts are given), the convolution's and the
    correlation's own times, and what they add to a step."""
    import numpy as np
    import torch
    from paper_2601_00551_amd import api, synth
    dev = torch.device("cuda:0")
    D, T = len(wl.array["qx"]), model.T
    fc, bw = synth.element_responses(D, np.random.default_rng(4000))
    m = api.with_response(ctx, model, torch.as_tensor(fc, device=dev), torch.as_tensor(bw, device=dev))
    gt = {k: torch.as_tensor(v, device=dev) for k, v in wl.init.items()}
    gt["p0"] = gt["p0"] * 1.5
    y_real = api.simulate_signals(ctx, A, gt, m)
    del gt
    rng = np.random.default_rng(3001)
    sigma = 0.05 * float(y_real.abs().max())
    y_real += sigma * torch.as_tensor(rng.normal(size=tuple(y_real.shape)).astype(np.float32), device=dev)
    cap = args.balls
    a = api.State(wl.init, capacity=cap, device=dev)
    b = api.State({k: np.zeros(0) for k in api.PARAMS}, ball_off=[0, 0], capacity=cap, device=dev)
    y_k = torch.empty_like(y_real)
    y_work = torch.empty_like(y_real)
    prm = api.AdamParams(lr=(0.005, 0.005, 0.005, 0.02, 0.002), step=1)
    rule = api.GrowthRule(destroy_frac=0.02, a_min=0.02, a_split=0.3, dup_frac=0.0)

    def one():
        api.downsample(ctx, y_real, 1, out=y_k)
        api.filter_zero_grad(ctx, A, a.balls, m, y_k, ball_off=a.ball_off, strict=True, out=b.balls,
                             off_out=b.ball_off, B_cap=a.B_cap, moments=(a.m, a.v), moments_out=(b.m, b.v))
        api.simulate_signals(ctx, A, b.balls, m, ball_off=b.ball_off, y=y_work, B_cap=b.B_cap)
        api.residual_loss(ctx, y_work, y_k, v_out=y_work)
        api.adjoint_gradients(ctx, A, b.balls, m, y_work, mask=api.ALL, ball_off=b.ball_off,
                              grad=b.grad, B_cap=b.B_cap)
        api.adam_update(ctx, b, prm)
        new, _ = api.grow(ctx, b, rule, capacity=cap)
        for k in api.PARAMS:
            a.balls[k], new.balls[k] = new.balls[k], a.balls[k]
            a.m[k], new.m[k] = new.m[k], a.m[k]
            a.v[k], new.v[k] = new.v[k], a.v[k]
        a.ball_off.copy_(new.ball_off)
        prm.step += 1

    for _ in range(args.warmup):
        one()
    n_in = [a.count()]
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.response_steps):
        one()
        n_in.append(a.count())
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.response_steps
    # the convolution and the correlation on their own, over the whole record
    h, zero = m.response, m.response_zero
    L = h.shape[1]
    times = {}
    for name, adj in (("convolve", False), ("correlate", True)):
        api.response_apply(ctx, h, zero, y_k, adjoint=adj, out=y_work)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            api.response_apply(ctx, h, zero, y_k, adjoint=adj, out=y_work)
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 10
    fmas = float(D) * T * L
    # per step the response adds one convolution (simulate) and two
    # correlations (filter reference, adjoint cotangent)
    added = times["convolve"] + 2 * times["correlate"]
    out = {"taps": L, "rows": D, "sampling_MHz": round(1.0 / model.dt), "steps": args.response_steps,
           "ms_per_step": ms, "pairs_per_s": float(np.mean(n_in[:-1])) * D / (ms * 1e-3),
           "balls_in_per_step": float(np.mean(n_in[:-1])), "kept_by_filter": int(b.ball_off[-1].item()),
           "added_ms_per_step": added, "added_fraction_of_plain_step": added / ms_plain}
    for name, t in times.items():
        out[name] = {"ms": t, "fma_per_launch": fmas, "achieved_TOPs": fmas / (t * 1e-3) / 1e12,
                     "frac": fmas / (t * 1e-3) / VALU_PEAK, "hbm_bytes": 8.0 * D * T,
                     "hbm_GBs": 8.0 * D * T / (t * 1e-3) / 1e9}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--balls", type=int, default=2_000_000)
    ap.add_argument("--cpu-sample", type=int, default=40000, help="balls in the oracle sample (0 = skip)")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2601_00551_amd", "tuning.json"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (the reference for HBM counters)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain reconstruction timing")
    ap.add_argument("--response-steps", type=int, default=3,
                    help="steps timed again with a transducer response per element (0 = skip)")
    ap.add_argument("--tiny", action="store_true",
                    help="only the tiny workload's per-iteration latency (eager vs graph)")
    ap.add_argument("--suite", action="store_true",
                    help="measure the other workloads instead (one JSON line each)")
    ap.add_argument("--rates", action="store_true",
                    help="only run the issue-rate microbenchmark (VALU, transcendental, LDS)")
    args = ap.parse_args()
    if args.suite or args.tiny:
        suite(args)
        return
    if args.rates:
        import subprocess
        exe = os.path.join(ROOT, "paper_2601_00551_amd", "rates", "sbp_rates")
        if not os.path.exists(exe):
            raise SystemExit("sbp_rates is not built: run __graft_entry__.build() first")
        sys.exit(subprocess.run([exe]).returncode)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, device="cuda:0")     # 1 GiB of float32
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is a design only, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2601_00551_amd import api, synth
    from paper_2601_00551_amd import autotune

    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    wl = synth.large_config(n_balls=args.balls)
    T, dt, c = wl.T, wl.dt, 1.5
    model = api.Model(c=c, dt=dt, T=T, f=1, profile=api.PROFILE_GAUSS, directivity=api.DIR_COS)
    tuned = autotune.apply_cached(ctx, args.tuning, model, len(wl.array["qx"]), args.balls)
    A = {k: torch.as_tensor(v, device=dev) for k, v in wl.array.items()}
    B = args.balls
    D = len(wl.array["qx"])

    # measured signal: the cloud with p0 scaled up by 1.5 (so that the filter
    # keeps it), plus 5 % noise; the estimate starts from p0 as drawn
    rng = np.random.default_rng(3000)
    gt = {k: torch.as_tensor(v, device=dev) for k, v in wl.init.items()}
    gt["p0"] = gt["p0"] * 1.5
    y_real = api.simulate_signals(ctx, A, gt, model)
    sigma = 0.05 * float(y_real.abs().max())
    y_real += sigma * torch.as_tensor(rng.normal(size=tuple(y_real.shape)).astype(np.float32), device=dev)
    del gt
    cap = B
    st = [api.State(wl.init, capacity=cap, device=dev), api.State({k: np.zeros(0) for k in api.PARAMS},
                                                                 ball_off=[0, 0], capacity=cap, device=dev)]
    y_k = torch.empty_like(y_real)
    y_work = torch.empty_like(y_real)
    g_buf = torch.empty(cap, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    rule = api.GrowthRule(destroy_frac=0.02, a_min=0.02, a_split=0.3, dup_frac=0.0)
    prm = api.AdamParams(lr=(0.005, 0.005, 0.005, 0.02, 0.002), step=1)
    names = ("downsample", "filter", "forward", "residual", "adjoint", "adam", "grow")
    times = {n: [] for n in names}
    counts = {"in": [], "kept": []}
    cur = 0

    def one_step(record):
        nonlocal cur
        a, b = st[cur], st[1 - cur]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record()
        api.downsample(ctx, y_real, 1, out=y_k)
        ev[1].record()
        # filter a -> b (balls and moments compacted, p0 kept)
        out, off_out, _, _ = api.filter_zero_grad(
            ctx, A, a.balls, model, y_k, ball_off=a.ball_off, strict=True, out=b.balls,
            off_out=b.ball_off, g_out=g_buf, B_cap=a.B_cap, moments=(a.m, a.v),
            moments_out=(b.m, b.v))
        ev[2].record()
        api.simulate_signals(ctx, A, b.balls, model, ball_off=b.ball_off, y=y_work, B_cap=b.B_cap)
        ev[3].record()
        api.residual_loss(ctx, y_work, y_k, v_out=y_work, loss=loss)
        ev[4].record()
        api.adjoint_gradients(ctx, A, b.balls, model, y_work, mask=api.ALL, ball_off=b.ball_off,
                              grad=b.grad, B_cap=b.B_cap)
        ev[5].record()
        api.adam_update(ctx, b, prm)
        ev[6].record()
        new, cnt = api.grow(ctx, b, rule, capacity=cap)
        ev[7].record()
        # the grown cloud becomes the next step's input (moments carried by grow)
        for k in api.PARAMS:
            st[cur].balls[k], new.balls[k] = new.balls[k], st[cur].balls[k]
            st[cur].m[k], new.m[k] = new.m[k], st[cur].m[k]
            st[cur].v[k], new.v[k] = new.v[k], st[cur].v[k]
        st[cur].ball_off.copy_(new.ball_off)
        prm.step += 1
        if record:
            torch.cuda.synchronize()
            for i, n in enumerate(names):
                times[n].append(ev[i].elapsed_time(ev[i + 1]))
            counts["kept"].append(int(b.ball_off[-1].item()))

    for _ in range(args.warmup):
        counts["in"].append(st[cur].count())
        one_step(True)
    for n in names:
        times[n].clear()
    counts["kept"].clear()
    n_in = [st[cur].count()]
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(True)
        n_in.append(st[cur].count())
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    pairs_in = float(np.mean(n_in[:-1])) * D
    value = pairs_in / (ms_step * 1e-3)

    avg = {n: float(np.mean(times[n])) for n in names}
    kept = float(np.mean(counts["kept"]))
    E = edges_per_pair(5.0 * 0.15, c * dt)
    per_pair = algorithmic_ops(E)
    pairs = {"forward": kept * D, "adjoint": kept * D, "filter": float(np.mean(n_in[:-1])) * D}
    kernels = {}
    for n in ("forward", "adjoint", "filter"):
        ach = pairs[n] * per_pair[n] / (avg[n] * 1e-3)
        kernels[n] = {"ms": round(avg[n], 4), "pairs": pairs[n], "ops_per_pair": per_pair[n],
                      "achieved_TOPs": ach / 1e12, "frac": ach / VALU_PEAK,
                      "traffic": measured_traffic(n)}
    f_comp = pairs["forward"] * per_pair["forward_as_computed"] / (avg["forward"] * 1e-3)
    kernels["forward"]["as_computed"] = {"ops_per_pair": per_pair["forward_as_computed"],
                                         "achieved_TOPs": f_comp / 1e12, "frac": f_comp / VALU_PEAK}
    lds = pairs["forward"] * E / (avg["forward"] * 1e-3)      # one LDS add per support edge
    kernels["forward"]["lds_atomics"] = {
        "per_pair": E, "achieved_per_s": lds, "peak_per_s": LDS_PEAK, "frac": lds / LDS_PEAK,
        "frac_of_random_address_rate": lds / (256 * 2.4e9 * LDS_U64_RANDOM),
        "frac_of_rotated_pattern_rate": lds / (256 * 2.4e9 * LDS_U64_FORWARD_ROTATED)}
    dominant = max(("forward", "adjoint", "filter"), key=lambda n: avg[n])
    achieved = kernels[dominant]["achieved_TOPs"] * 1e12
    fwd_adj = kept * D / ((avg["forward"] + avg["adjoint"]) * 1e-3)
    line = {
        "metric": "fwd+adjoint ball-detector pairs/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "balls": B, "transducers": D, "samples": T,
                   "sampling_MHz": round(1.0 / dt), "profile": "gauss", "directivity": "cos",
                   "step": "downsample+filter+simulate+residual+adjoint+adam+grow"},
        "kernel_ms": {n: round(avg[n], 4) for n in names},
        "fwd_adj_pairs_per_s": fwd_adj,
        "balls_kept_by_filter": kept,
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": achieved / 1e12,
                     "peak": VALU_PEAK / 1e12, "unit": "TOP/s", "frac": achieved / VALU_PEAK,
                     "traffic": measured_traffic(dominant), "traffic_unit": "bytes/launch"},
        "kernels": kernels,
        "tuning": tuned,
        "wall_s": wall,
    }
    if args.response_steps > 0:
        del st, y_work, y_k
        torch.cuda.empty_cache()
        line["response"] = response_leg(ctx, wl, A, model, args, ms_step)
    line["mlp"] = mlp_rates(ctx, dev)
    if not args.no_learned:
        line["learned_vs_plain"] = learned_vs_plain(ctx)
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(wl, {"c": c, "dt": dt, "T": T}, args.cpu_sample)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
