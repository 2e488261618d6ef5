#!/usr/bin/env python3
"""RK4 stages/s of the TT step-truncation solver for the Burgers-Hopf
characteristic-function PDE on one MI355X, mixed-precision form against
plain FP64.

Workload (the metric's configuration, precision form): d = 50 Fourier
modes, n = 128 grid points per mode on [-8, 8], nu = 0.01, rank cap 64,
relative truncation tolerance 1e-6, dt = 2e-4.  The operator application's
sketch contractions run in split-FP16x3 on the fp16 matrix cores (FP32
accumulation; --precision bf16x3 selects split-BF16x3, fp64 the plain
form); QR, SVD, the truncation test and all sums stay FP64.  Timing uses
the saturated regime: the input is a seeded random TT with every interior
rank at the cap (64), so every stage runs at the worst-case shapes of the
configuration.  One step = one RK4 step-truncation step (4 stages: four
sketched operator applications, their truncations, the stage combinations
and their truncations) followed by a pointwise read-out of 1024 entries.

Before timing, the GEMM launch shapes (tile and split-K factor) of one
step of each timed form are tuned by the library's autotuner (untimed
set-up; `--no-autotune` keeps the shape rule).

Prints one JSON line.  `value` is stages per second (4 per step) of the
selected form over the timed steps, with the input resident in device
memory; `fp64_reference` times the plain FP64 form the same way from the
same input.  `error_vs_fp64` gives the relative L2 distance to the FP64
form per stage from identical inputs (the stage derivative k after its
truncation, and the stage output y = f + c dt k) in the timed regime and
along a trajectory from the seeded Gaussian initial condition, plus whole
steps from identical inputs; the gate is 1e-5.  The last warm-up step is
profiled per kernel class (HIP events around every launch); the class with
the most time becomes the roofline kernel, and only its launches are timed
with events inside the timed region.  `roofline` divides its algorithmic
FLOPs (or bytes, for memory-bound kernels) by its event-timed duration and
compares with the MI355X peak: FP64 78.6 TFLOP/s for the FP64 matrix-core
GEMM and the FP64 vector kernels, 2.5 PFLOP/s dense fp16/bf16 for the split
GEMMs (counting the three 16-bit products per real product they execute),
8 TB/s HBM.  `cpu_baseline` is the CPU oracle (full-grid RK4
step-truncation) on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

D, N, LEN, NU, CAP, EPS, DT = 50, 128, 8.0, 0.01, 64, 1e-6, 2e-4
PEAK_F64_TFLOPS = 78.6  # FP64: matrix cores and vector units alike
PEAK_F16_TFLOPS = 2500.0  # dense fp16 / bf16 matrix cores
PEAK_HBM_GBS = 8000.0
GATE = 1e-5
PROFILE_EVERY = 4  # one in four launches of the roofline kernel is event-timed
PRECISIONS = {"fp64": 0, "bf16x3": 1, "fp16x3": 2, "fp32": 3}
PEAK_F32_TFLOPS = 157.3  # FP32 matrix cores


def cpu_baseline(seconds_target=20.0):
    """The CPU oracle timed on this host: full-grid truncation-aware RK4 at
    d = 4, n = 32 (the d = 50 grid has 128^50 points and cannot be formed)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import fullgrid, galerkin
    from paper_2403_04946_amd import inputs

    d, n, length, nu = 4, 32, 4.0, 0.05
    prob = fullgrid.Problem(galerkin.coefficient_B(d), galerkin.coefficient_D(d), nu, n, length)
    mu, sig = inputs.ic_params(d, 0)
    f = fullgrid.gaussian_ic(mu, sig, n, length)
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = fullgrid.truncated_rk4_step(f, 1e-3, prob.apply, 1e-12, 8)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds_target or steps >= 50:
            break
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    assert np.isfinite(f).all()
    return {
        "value": 4.0 * steps / el,
        "unit": "RK stages/s",
        "cores": int(threads),
        "host": host_info(),
        "kind": "oracle",
        "sample": (f"{steps} full-grid RK4 step-truncation steps (cap 8, eps 1e-12) at d=4, n=32 "
                   f"({el:.1f} s); the d=50, n=128 grid (128^50 points) cannot be formed on a CPU"),
    }


def host_info():
    """CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def gpu_oracle_workload(steps=20):
    """The oracle's workload on the GPU through the library (d = 4, n = 32,
    cap 8, eps 1e-12, dt 1e-3, exact apply, RK4 from the seeded Gaussian
    initial condition): stages/s beside the oracle's."""
    import torch

    from paper_2403_04946_amd import inputs, tt

    ctx = tt.Context(0)
    op = tt.Operator(ctx, 4, 32, 4.0, 0.05)
    f = tt.Tensor(ctx, 4, 32, 8)
    mu, sig = inputs.ic_params(4, 0)
    f.set_gaussian(mu, sig, 4.0)
    for _ in range(2):
        tt.tt_step(ctx, op, f, 1e-3, 8, 1e-12, tt.TT_APPLY_EXACT)
    f.set_gaussian(mu, sig, 4.0)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tt.tt_step(ctx, op, f, 1e-3, 8, 1e-12, tt.TT_APPLY_EXACT)
    ctx.sync()
    el = time.perf_counter() - t0
    op.close()
    f.close()
    ctx.close()
    return {"value": 4.0 * steps / el, "unit": "RK stages/s",
            "sample": f"{steps} RK4 step-truncation steps of the oracle's workload (d=4, n=32, cap 8) on the GPU"}


# kernel classes that are one kernel each, with the resource that bounds them
KERNEL_BOUND = {
    "zgemm": "mfma", "zgemm_fp16x3": "mfma", "zgemm_bf16x3": "mfma", "zgemm_fp32": "mfma", "chol_solve": "alu",
    "pt_leaf": "alu",
    "jacobi_cross": "alu", "jacobi_circle": "alu", "pt_assemble": "hbm", "panel_trmm": "hbm", "bcgs_pip": "alu",
    "gather_left": "hbm", "gather_right": "hbm", "zgemm_reduce": "hbm", "concat": "hbm",
}


# event counters of the library's statistics (no timing)
COUNTERS = {"qr_fallbacks", "jacobi_svds", "jacobi_sweeps_launched", "jacobi_sweeps_needed", "jacobi_check_passed"}


def dominant(stats):
    """The single-kernel class with the most time in a profiled step."""
    cand = {k: v["ms"] for k, v in stats.items() if k in KERNEL_BOUND}
    return max(cand, key=cand.get)


def roofline(name, kd, with_traffic=True):
    bound = KERNEL_BOUND[name]
    sec = kd["ms"] / 1e3
    if bound == "hbm":
        achieved, peak, unit, work = kd["bytes"] / sec / 1e9, PEAK_HBM_GBS, "GB/s", "bytes"
    else:
        peak = (PEAK_F16_TFLOPS if name in ("zgemm_fp16x3", "zgemm_bf16x3")
                else PEAK_F32_TFLOPS if name == "zgemm_fp32" else PEAK_F64_TFLOPS)
        achieved, unit, work = kd["flops"] / sec / 1e12, "TFLOP/s", "flops"
    return {
        "bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
        "traffic": traffic_per_launch(name) if with_traffic else None, "kernel": name, "launches": kd["launches"],
        "avg_launch_us": 1e3 * kd["ms"] / max(kd["launches"], 1),
        "algorithmic_flops_per_launch": kd["flops"] / max(kd["launches"], 1),
        "algorithmic_bytes_per_launch": kd["bytes"] / max(kd["launches"], 1),
        "work": work,
    }


def traffic_per_launch(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel, when one exists for the current source of the kernel."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(name)
    if not rec:
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), rec["source"])
    with open(src, "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != rec["sha256"]:
            return None
    return rec["bytes_per_launch"]


def rel_tt(ctx, tt, a, b):
    """||a - b|| / ||b|| of device TTs via the difference TT."""
    import numpy as np

    caps = np.array(a.ranks()) + np.array(b.ranks())
    caps[0] = caps[-1] = 1
    diff = tt.Tensor(ctx, D, N, caps)
    tt.tt_axpy(ctx, 1.0, a, -1.0, b, diff)
    r = tt.tt_norm(ctx, diff) / tt.tt_norm(ctx, b)
    diff.close()
    return r


def stage_errors(ctx, tt, op, f, prec, ell, seed, c=0.5 * DT, power=0):
    """One stage from the identical input f in FP64 and in `prec`: relative
    L2 of the truncated stage derivative k and of the stage output
    y = T[f + c k]."""
    out = {}
    ks = []
    for p in (0, prec):
        k = tt.Tensor(ctx, D, N, max(ell, CAP))
        tt.tt_apply(ctx, op, f, k, tt.TT_APPLY_SKETCH, ell, seed, precision=p, power=power)
        tt.tt_round(ctx, k, EPS, CAP, report=False)
        y = tt.Tensor(ctx, D, N, 2 * CAP)
        tt.tt_axpy(ctx, 1.0, f, c, k, y)
        tt.tt_round(ctx, y, EPS, CAP, report=False)
        ks.append((k, y))
    out["k"] = rel_tt(ctx, tt, ks[1][0], ks[0][0])
    out["stage_output"] = rel_tt(ctx, tt, ks[1][1], ks[0][1])
    for k, y in ks:
        k.close()
        y.close()
    return out


def error_report(ctx, tt, op, f0, prec, ell, traj_steps, power=0):
    """Errors of the `prec` form against plain FP64 from identical inputs:
    one stage and one step in the timed (saturated) regime, then along the
    FP64 trajectory from the seeded Gaussian initial condition every stage
    (from the FP64 stage input) and every step (from the FP64 step input)."""
    from paper_2403_04946_amd import inputs

    rep = {"gate": GATE}
    rep["saturated_stage"] = stage_errors(ctx, tt, op, f0, prec, ell, 99, power=power)
    a, b = tt.Tensor(ctx, D, N, CAP), tt.Tensor(ctx, D, N, CAP)
    a.copy_from(f0)
    b.copy_from(f0)
    tt.tt_step(ctx, op, a, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ell, 7, precision=0, power=power)
    tt.tt_step(ctx, op, b, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ell, 7, precision=prec, power=power)
    rep["saturated_step"] = rel_tt(ctx, tt, b, a)
    mu, sig = inputs.ic_params(D, 0)
    a.set_gaussian(mu, sig, LEN)
    ks, ys, steps = [], [], []
    for s in range(traj_steps):
        se = stage_errors(ctx, tt, op, a, prec, ell, 1000 + s, power=power)
        ks.append(se["k"])
        ys.append(se["stage_output"])
        b.copy_from(a)
        tt.tt_step(ctx, op, b, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ell, 500 + s, precision=prec, power=power)
        tt.tt_step(ctx, op, a, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ell, 500 + s, precision=0, power=power)
        steps.append(rel_tt(ctx, tt, b, a))
    rep["trajectory_from_ic"] = {"stage_k": ks, "stage_output": ys, "step": steps}
    worst = max([rep["saturated_stage"]["stage_output"], rep["saturated_step"]] + ys + steps)
    rep["worst_stage_output_or_step"] = worst
    rep["within_gate"] = bool(worst <= GATE)
    a.close()
    b.close()
    return rep


def main_batched(args):
    """Batched form: uneven independent instances (the batched workload's
    distribution: d uniform 8..64, n in {32, 64, 128}, nu log-uniform
    1e-3..1e-1, rank caps 16..96), each a seeded random TT with every
    interior rank at its cap, sketch width cap + 16 with one power pass,
    split-FP16x3 sketch pass, dt = 2e-4, eps = 1e-6.  The instances run in
    waves sized to HBM: ordered longest first by a cost estimate (d n cap^3)
    and packed greedily into waves of at most --wave instances whose
    estimated temporaries (45 x 16 d n cap^2 bytes each: the final RK4
    combination of rank 5 cap and its rounding) stay within --wave-gb; a
    wave steps all its instances concurrently by tt_step_batch, one context
    (host thread and stream) per instance, and frees them before the next.
    Instances of one wave have similar cost, so few wait on a straggler.
    The reference steps the instances of the first and the last wave one
    after another."""
    import torch

    from paper_2403_04946_amd import inputs, tt

    torch.cuda.init()
    specs = inputs.batch_instances(args.instances, 4)
    n = len(specs)
    cost = [sp["d"] * sp["n"] * sp["cap"] ** 3 for sp in specs]
    mem = [45 * 16 * sp["d"] * sp["n"] * sp["cap"] ** 2 for sp in specs]
    order = sorted(range(n), key=lambda i: -cost[i])
    waves, cur, cur_mem = [], [], 0
    for i in order:
        if cur and (len(cur) == args.wave or cur_mem + mem[i] > args.wave_gb * 1e9):
            waves.append(cur)
            cur, cur_mem = [], 0
        cur.append(i)
        cur_mem += mem[i]
    if cur:
        waves.append(cur)
    print(f"bench: {n} instances in {len(waves)} waves of {[len(w) for w in waves]}", file=sys.stderr, flush=True)

    def build(i):
        sp = specs[i]
        c = tt.Context(0)
        op = tt.Operator(c, sp["d"], sp["n"], 8.0, sp["nu"])
        f = tt.Tensor(c, sp["d"], sp["n"], sp["cap"])
        f.set_cores(inputs.random_tt(sp["d"], sp["n"], sp["cap"], sp["seed"]))
        return c, op, f

    def step(objs, sel):
        st = tt.tt_step_batch([objs[i][0] for i in sel], [objs[i][1] for i in sel], [objs[i][2] for i in sel],
                              [DT] * len(sel), [specs[i]["cap"] for i in sel], [EPS] * len(sel),
                              tt.TT_APPLY_SKETCH, [specs[i]["cap"] + 16 for i in sel], [specs[i]["seed"] for i in sel],
                              precision=tt.TT_PREC_FP16X3, power=args.sketch_power)
        if any(st):
            why = {i: tt.lib().tt_last_error(objs[i][0].h).decode() for i, v in zip(sel, st) if v}
            free, total = torch.cuda.mem_get_info()
            raise RuntimeError(f"batched step failed: {st} {why}; device memory free {free / 1e9:.1f} of "
                               f"{total / 1e9:.1f} GB")

    def release(objs):
        for c, op, f in objs.values():
            f.close()
            op.close()
            c.close()

    dom, tuned, tune_s = None, [], 0.0
    kd = {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "launches": 0}
    wave_s, seq_s = [], {}
    for wi, wave in enumerate(waves):
        objs = {i: build(i) for i in wave}
        for w in range(args.warmup):
            step(objs, wave)
        if dom is None:
            # the roofline kernel: the class with the most time in one batched
            # step of the first wave; tiles from the autotuner for its GEMM
            # shapes (untimed set-up)
            from paper_2403_04946_amd import autotune

            t0 = time.perf_counter()
            for c, _, _ in objs.values():
                c.reset_stats()
                c.set_profiling(True, shapes=True)
            step(objs, wave)
            shapes, classes = {}, {}
            for c, _, _ in objs.values():
                st = c.dump_stats()
                autotune.gemm_shapes(st, shapes)
                for k, v in st.items():
                    if k in KERNEL_BOUND:
                        classes.setdefault(k, {"ms": 0.0})["ms"] += v["ms"]
                c.set_profiling(False)
            dom = dominant(classes) if classes else "zgemm"
            if args.autotune:
                tuned = autotune.tune(objs[wave[0]][0], shapes, top=args.autotune_top or 64)
            tune_s = time.perf_counter() - t0
        for c, _, _ in objs.values():
            c.reset_stats()
            c.set_profile_filter(dom)
            c.set_profile_sampling(PROFILE_EVERY)
            c.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(args.steps):
            step(objs, wave)
        torch.cuda.synchronize()
        wave_s.append(time.perf_counter() - t0)
        for c, _, _ in objs.values():
            st = c.stats(dom)
            for k in kd:
                kd[k] += st[k]
            c.set_profiling(False)
            c.set_profile_filter(None)
            c.set_profile_sampling(1)
        if wi in (0, len(waves) - 1) and not args.no_sequential:
            t0 = time.perf_counter()
            for s_ in range(args.steps):
                for i in wave:
                    step(objs, [i])
            torch.cuda.synchronize()
            seq_s[wi] = time.perf_counter() - t0
        release(objs)
        print(f"bench: wave {wi + 1}/{len(waves)} ({len(wave)} instances) {wave_s[-1]:.1f} s", file=sys.stderr,
              flush=True)
    tb = sum(wave_s)
    stages = 4 * n * args.steps
    seq = {f"wave {wi + 1}": {"instances": len(waves[wi]), "batched_s": wave_s[wi], "sequential_s": t,
                              "speedup": t / wave_s[wi]} for wi, t in seq_s.items()}
    result = {
        "metric": "instance RK stages/sec, batched form",
        "value": stages / tb,
        "unit": "instance-stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * tb / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16x3+f64",
        "data": "synthetic",
        "config": {
            "workload": ("uneven independent Burgers-Hopf instances: d 8..64, n in {32,64,128}, nu 1e-3..1e-1, "
                         "caps 16..96, saturated ranks, split-FP16x3 sketch pass"),
            "instances": n, "dt": DT, "eps": EPS, "sketch_power": args.sketch_power,
            "waves": [len(w) for w in waves], "wave_limit": args.wave, "wave_gb": args.wave_gb,
            "instance_shapes": [[sp["d"], sp["n"], sp["cap"]] for sp in specs],
        },
        "wave_seconds": wave_s,
        "gemm_autotune": {"shapes_tuned": len(tuned), "seconds": tune_s},
        "sequential_reference": seq,
        # launches of the class from all instances overlap in time: the
        # figure is per launch (summed durations), not the chip's aggregate
        "roofline": roofline(dom, kd, with_traffic=False) if kd["launches"] else None,
    }
    print(json.dumps(result), flush=True)


def main_learned(args):
    """Learned form: the rank predictor (device MLP) trained on rank
    histories of plain trajectories, then held-out trajectories stepped in
    the plain and the learned form from the same initial condition.
    Instances: seeded Gaussian initial conditions, n = 64 on [-6, 6], nu
    log-uniform 0.02..0.1, rank cap 64, eps = 1e-6, dt = 5e-4, sketched
    apply of width 80 in FP64; training d uniform 6..16, held-out d 10..14.
    These are tolerance-limited trajectories (ranks below the cap); where the
    cap binds (the saturated metric shapes) the predicted ranks reach the
    cap and the step runs plain."""
    import numpy as np
    import torch

    from paper_2403_04946_amd import inputs, learned, tt

    torch.cuda.init()
    ctx = tt.Context(0)
    length, dt, eps, ell, cap = 12.0, 5e-4, 1e-6, 80, 64

    def instances(count, seed, d_range):
        return inputs.batch_instances(count, seed, d_range=d_range, n_choices=(64,), nu_range=(0.02, 0.1),
                                      cap_range=(cap, cap))

    def trajectory(inst, steps, predictor=None, seed=0):
        op = tt.Operator(ctx, inst["d"], inst["n"], length, inst["nu"])
        f = tt.Tensor(ctx, inst["d"], inst["n"], cap)
        f.set_gaussian(inst["mu"], inst["sigma"], length)
        recs = learned.run_trajectory(ctx, op, f, steps, dt, cap, eps, ell, inst["nu"], predictor=predictor,
                                      seed=seed)
        return op, f, recs

    t0 = time.perf_counter()
    xs, ys = [], []
    train = instances(args.train_instances, 21, (6, 16))
    for i, inst in enumerate(train):
        _, f, recs = trajectory(inst, args.train_steps)
        x, y = learned.samples_from_records(recs)
        xs.append(x)
        ys.append(y)
        f.close()
        print(f"bench: training trajectory {i + 1}/{len(train)} (d={inst['d']}) done", file=sys.stderr, flush=True)
    x, y = np.concatenate(xs), np.concatenate(ys)
    capture_s = time.perf_counter() - t0
    pred = learned.RankPredictor(ctx, cap, max_batch=max(4096, x.shape[0]), seed=1)
    t0 = time.perf_counter()
    l0, l1 = pred.fit(x, y)
    train_s = time.perf_counter() - t0
    print(f"bench: predictor trained on {x.shape[0]} samples", file=sys.stderr, flush=True)

    def rel_tt(a, b):
        aa, bb, ab = tt.tt_dot(ctx, a, a).real, tt.tt_dot(ctx, b, b).real, tt.tt_dot(ctx, a, b).real
        return float(np.sqrt(max(aa + bb - 2 * ab, 0.0) / bb))

    held = instances(args.instances_learned, 77, (10, 14))
    # the roofline kernel: the class with the most time in one profiled plain
    # step of the first held-out instance; during the held-out trajectories
    # (plain and learned alike) one launch in PROFILE_EVERY of it is
    # event-timed, and the learned ones' launches make the roofline
    op_p, f_p, _ = trajectory(held[0], 1)
    ctx.reset_stats()
    ctx.set_profiling(True)
    tt.tt_step(ctx, op_p, f_p, dt, cap, eps, tt.TT_APPLY_SKETCH, ell, 1)
    dom = dominant(ctx.dump_stats())
    ctx.set_profiling(False)
    f_p.close()
    ctx.set_profile_filter(dom)
    ctx.set_profile_sampling(PROFILE_EVERY)
    kd = {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "launches": 0}
    tp = tl = 0.0
    used = fb = afb = aused = 0
    diffs, rank_err = [], []
    for i, inst in enumerate(held):
        ctx.set_profiling(True)
        _, fp, plain = trajectory(inst, args.steps + 1, seed=3)
        ctx.reset_stats()
        _, fl, lrn = trajectory(inst, args.steps + 1, predictor=pred, seed=3)
        st = ctx.stats(dom)
        for k in kd:
            kd[k] += st[k]
        ctx.set_profiling(False)
        # the first step of either has no report to predict from: untimed
        tp += sum(r["wall"] for r in plain[1:])
        tl += sum(r["wall"] for r in lrn[1:])
        used += sum(r["learned_used"] for r in lrn)
        fb += sum(r["learned_fallback"] for r in lrn)
        afb += sum(r["apply_fallback"] for r in lrn)
        aused += sum(1 for r in lrn if r["apply_widths"] is not None)
        diffs.append(rel_tt(fl, fp))
        xt, yt = learned.samples_from_records(plain)
        rank_err.append(float(np.abs(pred.predict(xt) - yt).mean()))
        fp.close()
        fl.close()
        print(f"bench: held-out instance {i + 1}/{len(held)} (d={inst['d']}) done", file=sys.stderr, flush=True)
    stages = 4 * args.steps * len(held)
    result = {
        "metric": "RK stages/sec, learned form vs plain (deterministic rounding) on the same trajectories",
        "value": stages / tl,
        "unit": "RK stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": 1e3 * tl / (args.steps * len(held)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("Burgers-Hopf TT RK4 trajectories from seeded Gaussian initial conditions, tolerance-"
                         "limited ranks: n=64 on [-6,6], nu 0.02..0.1, cap 64, eps 1e-6, dt 5e-4, sketched "
                         "apply width 80, FP64; held-out d 10..14"),
            "held_out_shapes": [[h["d"], h["n"], cap] for h in held],
            "training": {"instances": len(train), "d_range": [6, 16], "steps": args.train_steps,
                         "samples": int(x.shape[0]), "loss_before": l0, "loss_after": l1,
                         "capture_s": capture_s, "train_s": train_s},
        },
        "plain_reference": {"value": stages / tp, "unit": "RK stages/s", "ms_per_step":
                            1e3 * tp / (args.steps * len(held))},
        "gain_over_plain": tp / tl,
        "randomised_roundings": used,
        "fallbacks": fb,
        "steps_with_learned_apply_widths": aused,
        "stage_applications_redone": afb,
        "rel_diff_to_plain_after_steps": diffs,
        "predictor_mean_abs_rank_error": rank_err,
        "learned_tol": 1e-6,
        "roofline": roofline(dom, kd, with_traffic=False) if kd["launches"] else None,
    }
    pred.close()
    print(json.dumps(result), flush=True)


def main_learned_full(args):
    """Learned form at its own configuration: the predictor trained on
    bond-step samples of plain trajectories at seeded d in 20..80 (n=64 on
    [-6, 6], cap 64, eps 1e-6, dt 5e-4, nu log-uniform 0.005..0.1), then a
    trajectory at d=100, n=128 on [-8, 8], nu=0.005, cap 128, eps 1e-6,
    dt 2e-4 from the seeded Gaussian IC, stepped plain and learned.  Per
    step it records the share of bonds whose rank sits at the cap (there the
    rounding is cap-limited and the learned form runs plain), the
    predictor's rank error, the randomised roundings tried and accepted,
    the largest sketch estimate of their error, and the step times."""
    import numpy as np
    import torch

    from paper_2403_04946_amd import inputs, learned, tt

    torch.cuda.init()
    ctx = tt.Context(0)
    ell = 80
    t0 = time.perf_counter()
    xs, ys = [], []
    train = inputs.batch_instances(args.train_instances, 31, d_range=(20, 80), n_choices=(64,),
                                   nu_range=(0.005, 0.1), cap_range=(64, 64))
    for i, inst in enumerate(train):
        op = tt.Operator(ctx, inst["d"], 64, 6.0, inst["nu"])
        f = tt.Tensor(ctx, inst["d"], 64, 64)
        f.set_gaussian(inst["mu"], inst["sigma"], 6.0)
        recs = learned.run_trajectory(ctx, op, f, args.train_steps, 5e-4, 64, 1e-6, ell, inst["nu"], seed=i)
        x, y = learned.samples_from_records(recs)
        xs.append(x)
        ys.append(y)
        f.close()
        op.close()
        print(f"bench: training trajectory {i + 1}/{len(train)} (d={inst['d']}, {x.shape[0]} samples) done",
              file=sys.stderr, flush=True)
    x, y = np.concatenate(xs), np.concatenate(ys)
    capture_s = time.perf_counter() - t0
    # targets are rank / cap: the network trained at cap 64 predicts a share
    # of the cap, read at the evaluation's cap 128
    pred = learned.RankPredictor(ctx, 64, max_batch=max(4096, x.shape[0]), seed=1)
    t0 = time.perf_counter()
    l0, l1 = pred.fit(x, y)
    train_s = time.perf_counter() - t0
    print(f"bench: predictor trained on {x.shape[0]} samples", file=sys.stderr, flush=True)
    pred.rmax = 128
    d, n, length, nu, cap, eps, dt = 100, 128, 8.0, 0.005, 128, 1e-6, 2e-4
    mu, sig = inputs.ic_params(d, 5)
    out = {}
    for form in ("plain", "learned"):
        op = tt.Operator(ctx, d, n, length, nu)
        f = tt.Tensor(ctx, d, n, cap)
        f.set_gaussian(mu, sig, length)
        steps = []

        def note(s, rec):
            inner = rec["ranks"][1:-1]
            steps.append({"step": s + 1, "wall_s": rec["wall"], "max_rank": max(inner),
                          "bonds_at_cap": sum(1 for r in inner if r >= cap) / len(inner),
                          "widths_predicted": rec["widths"] is not None,
                          "randomised_roundings": rec["learned_used"], "fallbacks": rec["learned_fallback"],
                          "largest_estimate": rec["learned_err"]})
            print(f"bench: {form} d=100 step {s + 1}: max rank {max(inner)}, "
                  f"{steps[-1]['bonds_at_cap']:.2f} of the bonds at the cap, {rec['wall']:.1f} s",
                  file=sys.stderr, flush=True)

        recs = learned.run_trajectory(ctx, op, f, args.steps, dt, cap, eps, ell, nu,
                                      predictor=pred if form == "learned" else None, seed=3, on_step=note)
        if form == "plain":
            xt, yt = learned.samples_from_records(recs)
            rank_err = float(np.abs(pred.predict(xt) - yt).mean()) if xt.shape[0] else None
        out[form] = steps
        f.close()
        op.close()
    result = {
        "form": "learned, full configuration",
        "training": {"instances": len(train), "d_range": [20, 80], "n": 64, "cap": 64, "steps": args.train_steps,
                     "samples": int(x.shape[0]), "loss_before": l0, "loss_after": l1, "capture_s": capture_s,
                     "train_s": train_s},
        "evaluation": {"d": d, "n": n, "L": length, "nu": nu, "cap": cap, "eps": eps, "dt": dt,
                       "sketch_width": ell, "predictor_mean_abs_rank_error": rank_err},
        "plain": out["plain"], "learned": out["learned"], "learned_tol": 1e-6,
    }
    pred.close()
    print(json.dumps(result), flush=True)


TRAJECTORIES = {
    # d, n, L, nu, cap, eps, dt, sketch width
    "d20": (20, 64, 6.0, 0.02, 32, 1e-8, 5e-4, 80),
    "d50": (50, 128, 8.0, 0.01, 64, 1e-6, 2e-4, 80),
}


def main_trajectory(args):
    """A trajectory from the initial condition (Sec. 4.1 explicit RK4
    step-truncation, which has a time-step restriction), logged per step:
    bond ranks, ||phi||, phi at the origin's nearest node, the largest
    |phi| over 4096 sampled nodes and the step time.  The run stops when a
    sampled |phi| exceeds 1 + phi_tol (a characteristic function is bounded
    by 1), ||phi|| exceeds `growth` times its initial value or stops being
    finite: the explicit scheme has become unstable.  Workloads: d20 (n=64 on
    [-6, 6], nu 0.02, cap 32, eps 1e-8, dt 5e-4; Gaussian or rank-3
    tridiagonal-covariance IC) and d50 (n=128 on [-8, 8], nu 0.01, cap 64,
    eps 1e-6, dt 2e-4).  One JSON line per step to --log, a summary line to
    stdout."""
    import numpy as np
    import torch

    from paper_2403_04946_amd import inputs, tt

    torch.cuda.init()
    d, n, length, nu, cap, eps, dt, ell = TRAJECTORIES[args.trajectory]
    if args.dt:
        dt = args.dt
    prec = PRECISIONS[args.precision]
    ctx = tt.Context(0)
    op = tt.Operator(ctx, d, n, length, nu)
    f = tt.Tensor(ctx, d, n, cap)
    if args.ic == "tridiag":
        mu, sig, rho = inputs.ic_params_tridiag(d, 0)
        ic_rep = f.set_gaussian_tridiag(mu, sig, rho, length, 0.0, 3)
        ic_tail = max(ic_rep["tail"]) / ic_rep["norm"]
    else:
        mu, sig = inputs.ic_params(d, 0)
        f.set_gaussian(mu, sig, length)
        ic_tail = 0.0
    idx = inputs.random_points(d, n, 4096, 3)
    idx[0] = n // 2  # the node next to the origin
    idx_d = torch.from_numpy(idx).cuda()
    out = torch.empty(4096, dtype=torch.complex128, device="cuda")
    norm0 = tt.tt_norm(ctx, f)
    log = open(args.log, "w") if args.log else None
    t0 = time.perf_counter()
    status, last = "completed", None
    for s in range(1, args.steps + 1):
        ts = time.perf_counter()
        rep = tt.tt_step(ctx, op, f, dt, cap, eps, tt.TT_APPLY_SKETCH, ell, 1000 + s, precision=prec,
                         power=args.sketch_power)
        tt.tt_eval(ctx, f, idx_d, out)
        v = out.cpu().numpy()
        nrm = tt.tt_norm(ctx, f)
        rec = {"step": s, "t": s * dt, "max_rank": max(f.ranks()), "norm": nrm, "norm_ratio": nrm / norm0,
               "phi_origin_node": [float(v[0].real), float(v[0].imag)], "max_abs_sampled": float(np.abs(v).max()),
               "step_s": time.perf_counter() - ts, "step_max_rank": rep["max_rank"]}
        last = rec
        if log:
            log.write(json.dumps(rec) + "\n")
            log.flush()
        if s % 10 == 0 or s == 1:
            print(f"bench: trajectory step {s}: rank {rec['max_rank']}, |phi| ratio {rec['norm_ratio']:.6f}, "
                  f"max sampled |phi| {rec['max_abs_sampled']:.6f}", file=sys.stderr, flush=True)
        if not np.isfinite(nrm) or nrm > args.growth * norm0 or rec["max_abs_sampled"] > 1.0 + args.phi_tol:
            status = (f"unstable at step {s}: ||phi|| / ||phi0|| = {nrm / norm0:.3e}, "
                      f"max sampled |phi| = {rec['max_abs_sampled']:.3e}")
            break
        if time.perf_counter() - t0 > args.max_seconds:
            status = f"stopped at the time limit after step {s}"
            break
    result = {"form": "trajectory", "workload": args.trajectory, "ic": args.ic, "precision": args.precision,
              "sketch_width": ell, "sketch_power": args.sketch_power,
              "d": d, "n": n, "L": length, "nu": nu, "rank_cap": cap, "eps": eps, "dt": dt,
              "ic_discarded_tail": ic_tail, "norm0": norm0, "status": status, "last": last,
              "wall_s": time.perf_counter() - t0}
    print(json.dumps(result), flush=True)


def main_cdf(args):
    """The paper's own workload: the CDF equation of the stochastic Burgers
    equation with reaction (Sec. 5) at N = 20 points of the circle, n = 64
    points per phase variable on [-1.3, 1.3], explicit midpoint
    step-truncation (the paper's integrator) at TT ranks above 100: a seeded
    random TT with every interior rank 128 (cap 128), sketched apply of
    width 144, eps 1e-8, dt 1e-3, gamma 0.05, alpha 1 (the paper states
    neither coefficient), all in FP64 (complex storage; the CDF is real).
    Reported beside the paper's figure for the same size on its CPU
    workstation (about 45 minutes per step at ranks above 100)."""
    import torch

    from paper_2403_04946_amd import inputs, tt

    torch.cuda.init()
    d, n, box, cap, ell, eps, dt = 20, 64, 1.3, 128, 144, 1e-8, 1e-3
    ctx = tt.Context(0)
    op = tt.CdfOperator(ctx, d, n, box, 0.05, 1.0)
    f0 = tt.Tensor(ctx, d, n, cap)
    f0.set_cores(inputs.random_tt(d, n, cap, 0))
    f = tt.Tensor(ctx, d, n, cap)
    f.copy_from(f0)

    def step():
        return tt.tt_step(ctx, op, f, dt, cap, eps, tt.TT_APPLY_SKETCH, ell, 7, scheme=tt.TT_STEP_MIDPOINT)

    breakdown = None
    for i in range(args.warmup):
        if i == args.warmup - 1:
            ctx.reset_stats()
            ctx.set_profiling(True)
        step()
        f.copy_from(f0)
        if i == args.warmup - 1:
            breakdown = ctx.dump_stats()
            ctx.set_profiling(False)
        print(f"bench: CDF warm-up step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.sync()
    dom = dominant(breakdown) if breakdown else "zgemm"
    ctx.reset_stats()
    ctx.set_profile_filter(dom)
    ctx.set_profile_sampling(PROFILE_EVERY)
    ctx.set_profiling(True)
    stream = ctx.torch_stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    rep = None
    for _ in range(args.steps):
        rep = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kd = ctx.stats(dom)
    ctx.set_profiling(False)
    ctx.set_profile_filter(None)
    ctx.set_profile_sampling(1)
    print("bench: CDF timed steps done", file=sys.stderr, flush=True)
    sec = ms / 1e3 / args.steps
    paper_sec = 45 * 60.0
    result = {
        "metric": "seconds per explicit-midpoint step, CDF equation N=20, n=64, TT ranks 128",
        "value": sec,
        "unit": "s/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("CDF equation of the stochastic Burgers equation with reaction, explicit midpoint "
                         "step-truncation, N=20, n=64 on [-1.3,1.3], gamma 0.05, alpha 1, cap 128, eps 1e-8, "
                         "dt 1e-3, sketched apply width 144, FP64; input a seeded random TT with interior ranks 128"),
            "stage_max_rank": rep["max_rank"] if rep else None,
            "final_ranks_max": max(f.ranks()),
        },
        "paper_context": {"seconds_per_step": paper_sec, "hardware": "Intel i9-7980XE workstation (CPU)",
                          "ranks": "above 100", "speedup_of_this_run": paper_sec / sec},
        "roofline": roofline(dom, kd, with_traffic=False),
        "kernels_ms_profiled_warmup_step": {k: round(v["ms"], 3) for k, v in (breakdown or {}).items()
                                            if k not in COUNTERS},
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sketch-rank", type=int, default=80)
    ap.add_argument("--sketch-power", type=int, default=1,
                    help="subspace-iteration passes of every sketched apply (0 = the plain range finder)")
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default="fp16x3")
    ap.add_argument("--mixed-passes", type=int, choices=(0, 1), default=1,
                    help="1: the reduced precision in every pass of the sketched apply but the last (0: in the "
                         "Gaussian sketch pass only)")
    ap.add_argument("--error-steps", type=int, default=2,
                    help="trajectory steps from the initial condition in the error report")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-error-report", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", choices=["metric", "batched", "learned", "learned-full", "cdf", "trajectory"],
                    default="metric",
                    help="batched: the batched form on uneven instances; learned: the learned form against the "
                         "plain one on tolerance-limited trajectories; trajectory: a logged run from the initial "
                         "condition (each its own JSON line)")
    ap.add_argument("--trajectory", choices=sorted(TRAJECTORIES), default="d20")
    ap.add_argument("--ic", choices=["gaussian", "tridiag"], default="gaussian")
    ap.add_argument("--dt", type=float, default=None, help="trajectory: time step (default: the workload's)")
    ap.add_argument("--log", default=None, help="trajectory: per-step JSON lines to this file")
    ap.add_argument("--growth", type=float, default=1e3,
                    help="trajectory: stop when ||phi|| exceeds this multiple of its initial value")
    ap.add_argument("--phi-tol", type=float, default=1e-3,
                    help="trajectory: stop when a sampled |phi| exceeds 1 + this (a characteristic function "
                         "has |phi| <= 1; the grid L2 norm itself grows as the distribution concentrates)")
    ap.add_argument("--max-seconds", type=float, default=240.0, help="trajectory: wall-clock limit")
    ap.add_argument("--instances", type=int, default=16)
    ap.add_argument("--wave", type=int, default=16, help="batched: instances per wave at most")
    ap.add_argument("--wave-gb", type=float, default=200.0,
                    help="batched: estimated temporaries per wave at most (GB)")
    ap.add_argument("--no-sequential", action="store_true", help="batched: skip the one-after-another reference")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the GEMM launch-shape rule (by default the shapes of one step of each timed form "
                         "are tuned before timing)")
    ap.add_argument("--autotune-top", type=int, default=None,
                    help="GEMM shapes tuned, heaviest first (default: 200, every shape of a step, for the "
                         "metric form; 64 for the batched form)")
    ap.add_argument("--autotune-save", default=None, help="write the tuned GEMM table (JSON) at the end")
    ap.add_argument("--autotune-load", default=None, help="use this GEMM table instead of tuning")
    ap.add_argument("--train-instances", type=int, default=12)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--instances-learned", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.form == "batched":
        # more hardware queues than the default 4, so the contexts' streams
        # do not share queues (set before the HIP runtime starts)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")
        main_batched(args)
        return
    if args.form == "learned":
        main_learned(args)
        return
    if args.form == "learned-full":
        main_learned_full(args)
        return
    if args.form == "cdf":
        main_cdf(args)
        return
    if args.form == "trajectory":
        main_trajectory(args)
        return

    import torch

    from paper_2403_04946_amd import inputs, tt

    torch.cuda.init()
    ctx = tt.Context(0)
    ctx.set_option(tt.TT_OPT_SKETCH_MIXED_PASSES, args.mixed_passes)
    op = tt.Operator(ctx, D, N, LEN, NU)
    prec = PRECISIONS[args.precision]
    f0 = tt.Tensor(ctx, D, N, CAP)
    f0.set_cores(inputs.random_tt(D, N, CAP, 0))
    f = tt.Tensor(ctx, D, N, CAP)
    f.copy_from(f0)
    idx = torch.from_numpy(inputs.random_points(D, N, 1024, 1)).cuda()
    out = torch.empty(1024, dtype=torch.complex128, device="cuda")
    ell = args.sketch_rank
    power = args.sketch_power
    seed = 12345

    def step(p=prec):
        rep = tt.tt_step(ctx, op, f, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ell, seed, precision=p, power=power)
        tt.tt_eval(ctx, f, idx, out)
        return rep

    tuned = None
    if args.autotune_load:
        # a table written by an earlier run (--autotune-save)
        from paper_2403_04946_amd import autotune

        autotune.load(args.autotune_load)
        tuned = {"loaded": args.autotune_load, "entries": len(tt.gemm_table())}
        args.autotune = False
    elif args.autotune:
        # GEMM launch shapes of one step, the heaviest tuned (untimed set-up)
        from paper_2403_04946_amd import autotune

        t0 = time.perf_counter()
        shapes = autotune.profile_shapes(ctx, step)
        res = autotune.tune(ctx, shapes, top=args.autotune_top or 200)
        tuned = {"shapes_tuned": len(res), "seconds": time.perf_counter() - t0}
        print(f"bench: autotuned {len(res)} GEMM shapes", file=sys.stderr, flush=True)
    # warm-up; the last warm-up step is profiled per kernel class to find
    # the dominant kernel, whose launches alone are then timed with HIP
    # events inside the timed region (so the step time carries the event
    # overhead of that class only)
    breakdown = None
    for i in range(args.warmup):
        if i == args.warmup - 1:
            ctx.reset_stats()
            ctx.set_profiling(True)
        step()
        if i == args.warmup - 1:
            breakdown = ctx.dump_stats()
            ctx.set_profiling(False)
        print(f"bench: warm-up step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.sync()
    torch.cuda.synchronize()
    dom = dominant(breakdown) if breakdown else "zgemm"
    ctx.reset_stats()
    ctx.set_profile_filter(dom)
    ctx.set_profile_sampling(PROFILE_EVERY)
    ctx.set_profiling(True)
    stream = ctx.torch_stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    rep = None
    for _ in range(args.steps):
        rep = step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    print(f"bench: {args.steps} timed steps done", file=sys.stderr, flush=True)
    ms = e0.elapsed_time(e1)
    kd = ctx.stats(dom)
    ctx.set_profiling(False)
    ctx.set_profile_filter(None)
    ctx.set_profile_sampling(1)
    assert torch.isfinite(out.real).all() and torch.isfinite(out.imag).all()

    stages = 4 * args.steps
    value = stages / (ms / 1e3)
    final_ranks_max = max(f.ranks())

    fp64_ref = None
    if prec != 0 and not args.no_fp64_reference:
        # the plain FP64 form from the same input, timed the same way (its
        # own GEMM shapes tuned first, like the selected form's)
        f.copy_from(f0)
        if args.autotune:
            from paper_2403_04946_amd import autotune

            autotune.tune(ctx, autotune.profile_shapes(ctx, lambda: step(0)), top=args.autotune_top or 200)
            f.copy_from(f0)
        step(0)
        ctx.sync()
        torch.cuda.synchronize()
        f.copy_from(f0)
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for _ in range(args.steps):
            step(0)
        r1.record(stream)
        torch.cuda.synchronize()
        ms64 = r0.elapsed_time(r1)
        fp64_ref = {"value": stages / (ms64 / 1e3), "unit": "RK stages/s", "ms_per_step": ms64 / args.steps,
                    "speedup_of_selected_form": (stages / (ms / 1e3)) / (stages / (ms64 / 1e3))}
        print(f"bench: FP64 reference, {args.steps} timed steps done", file=sys.stderr, flush=True)
    errors = None
    if prec != 0 and not args.no_error_report:
        errors = error_report(ctx, tt, op, f0, prec, ell, args.error_steps, power=power)
        print("bench: error report done", file=sys.stderr, flush=True)
    if args.autotune_save:
        from paper_2403_04946_amd import autotune

        autotune.save(args.autotune_save)
    roof = roofline(dom, kd)
    kernels_ms = {k: round(v["ms"], 3) for k, v in (breakdown or {}).items() if k not in COUNTERS}
    # per kernel class of the profiled warm-up step: launches and the
    # algorithmic rates over its event-timed duration (profiling included)
    kernel_rates = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                        "tflops": round(v["flops"] / (v["ms"] * 1e9), 3) if v["ms"] > 0 and v["flops"] > 0 else None,
                        "gbps": round(v["bytes"] / (v["ms"] * 1e6), 1) if v["ms"] > 0 and v["bytes"] > 0 else None}
                    for k, v in (breakdown or {}).items() if k not in COUNTERS}
    result = {
        "metric": "RK stages/sec at d=50,n=128,r<=64 vs plain FP64 at rel-L2 err <=1e-5",
        "value": value,
        "unit": "RK stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f64", 1: "bf16x3+f64", 2: "fp16x3+f64", 3: "fp32+f64"}[prec],
        "data": "synthetic",
        "config": {
            "workload": ("Burgers-Hopf TT RK4 step-truncation, saturated ranks, "
                         + {0: "plain complex FP64",
                            1: "sketch contractions split-BF16x3 (FP32 accumulate), QR/SVD/truncation FP64",
                            2: "sketch contractions split-FP16x3 (FP32 accumulate), QR/SVD/truncation FP64",
                            3: "sketch contractions FP32 (FP32 matrix cores, FP64 across K steps), "
                               "QR/SVD/truncation FP64"}[prec]),
            "precision": args.precision,
            "d": D, "n": N, "L": LEN, "nu": NU, "rank_cap": CAP, "eps": EPS, "dt": DT,
            "apply": f"sketched (width {ell}, {power} subspace-iteration passes)",
            "sketch_width": ell, "sketch_power": power,
            "input": "seeded random TT, all interior ranks 64",
        },
        "roofline": roof,
        "fp64_reference": fp64_ref,
        "error_vs_fp64": errors,
        "kernels_ms_profiled_warmup_step": kernels_ms,
        "kernel_rates_profiled_warmup_step": kernel_rates,
        "qr_fallbacks": int((breakdown or {}).get("qr_fallbacks", {"launches": 0})["launches"]),
        "jacobi_profiled_warmup_step": {k: int((breakdown or {}).get(k, {"launches": 0})["launches"])
                                        for k in sorted(COUNTERS) if k.startswith("jacobi_")},
        "wall_s": wall,
        "gemm_autotune": tuned,
        "final_ranks_max": final_ranks_max,
        "step_max_rank": rep["max_rank"] if rep else None,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline()
        result["cpu_baseline"]["gpu_same_workload"] = gpu_oracle_workload()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
