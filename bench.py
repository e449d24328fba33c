#!/usr/bin/env python3
"""Throughput of the WMC-regularised denoising solver on one MI355X.

One "step" is one whole solve of the plain WMC denoising problem on the
4096 x 4096 fp32 workload: 200 Jacobi updates
U <- U + dt[(f - U) + lam H_d(U)] (lam = 1, default dt = 1/(1+lam)), every
update evaluating the Half Laplace Operator at every pixel, from U^0 = f, with
f and the state resident in HBM.  The library fuses several updates per pass
over memory (temporal blocking) and replays the launch sequence as a hipGraph.

Printed: one JSON line with the metric (Gpixel-iterations/s), the roofline
of the dominant kernel measured with HIP events on the stream the graph runs
on, the FP64 CPU oracle timed on bounded samples, and extras: the plain
single-update kernel's HBM bandwidth (warm, cold and at 8192^2), the operator
alone, the differentiable 16 x 512^2 solve's training step, and the
uneven-size batched solve against per-image plain launches.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpixel-iter/s of WMC step (fp32) and % HBM roofline; batched vs per-image"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # lane-ops/s: 256 CUs x 4 SIMD16 x 2.4 GHz = 39.3
# Arithmetic of one pixel update in the column-sum form (wmc_device.hpp):
# row quantities 3 + odd/even parts 10 + candidates 8 + selection 14 + update 3.
ALGO_OPS_PER_PX_ITER = 38
BYTES_PER_PX_PASS = 12         # read U and f, write U' once per pass over memory


def depths(iters: int, T: int):
    """Launch depths the library uses for `iters` sweeps at maximum depth T."""
    out = []
    allowed = (8, 6, 4, 3, 2, 1)
    while iters > 0:
        t = min(iters, T)
        t = next(d for d in allowed if d <= t)
        out.append(t)
        iters -= t
    return out


def kernel_sha():
    h = hashlib.sha256()
    for name in ("wmc_stream.hip", "wmc_device.hpp"):
        with open(os.path.join(ROOT, "paper_1903_07189_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(tuning, side):
    """Bytes per launch leaving L2 (FETCH_SIZE + WRITE_SIZE, calibrated; the
    Infinity Cache's hits included) from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and this launch
    shape (lines "- hbm_bytes_per_launch[C,T,R]: N"); else None."""
    path = os.path.join(ROOT, "profiles", f"stream_kernel_{side}_counters.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_sha") != kernel_sha():
        return None
    key = f"hbm_bytes_per_launch[{tuning['cols']},{tuning['tsteps']},{tuning['seg_rows']}]"
    try:
        return float(kv[key]) if key in kv else None
    except ValueError:
        return None


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo, as lscpu reports it)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(side: int, sample_iters: int):
    """The FP64 oracle (single thread, pinned to one core) on the same input."""
    import numpy as np
    import oracle
    import wmc_synth
    try:
        cpus = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {sorted(cpus)[0]})
    except (AttributeError, OSError):
        cpus = None
    noisy, _ = wmc_synth.c2(side=side)
    f = noisy[0].astype(np.float64)
    t0 = time.perf_counter()
    oracle.solve(f, lam=1.0, iters=sample_iters)
    dt = time.perf_counter() - t0
    out = {"value": round(side * side * sample_iters / dt / 1e9, 6), "unit": "Gpixel-iter/s",
           "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
           "host_logical_cpus": len(cpus) if cpus else os.cpu_count(),
           "sample": f"{side}x{side} input, {sample_iters} of the 200 iterations "
                     f"({dt:.1f} s, FP64, one thread)"}
    # two more bounded samples: the 256 x 256 parity image in full (50
    # iterations) and one 512 x 512 image of the differentiable workload,
    # forward + adjoint of K = 20 steps
    c1, _ = wmc_synth.c1()
    t0 = time.perf_counter()
    oracle.solve(c1[0], lam=1.0, iters=50)
    t_c1 = time.perf_counter() - t0
    c4, _ = wmc_synth.c4(batch=1)
    g = np.random.default_rng(0).standard_normal((512, 512))
    t0 = time.perf_counter()
    oracle.solve_adjoint(g, f=c4[0, 0], lam=1.0, K=20)
    t_c4 = time.perf_counter() - t0
    out["samples"] = {"c1_256_50_iters_s": round(t_c1, 3),
                      "c1_gpx_iter_s": round(256 * 256 * 50 / t_c1 / 1e9, 6),
                      "c4_one_image_fwd_adjoint_s": round(t_c4, 3)}
    if cpus:
        os.sched_setaffinity(0, cpus)  # the aggregate sample uses every core
    out["aggregate"] = aggregate_oracle()
    return out


def _oracle_job(args):
    b, h, w, sig, iters = args
    import time as _t
    import oracle
    import wmc_synth
    noisy, _ = wmc_synth.c3_image(b, h, w, sig)
    t0 = _t.perf_counter()
    oracle.solve(noisy[0], lam=1.0, iters=iters)
    return h * w * iters, _t.perf_counter() - t0


def aggregate_oracle(max_procs: int = 16, iters: int = 2):
    """Host throughput with one oracle process per core on the uneven batch
    (first channel of the first `procs` images, `iters` iterations each):
    the sum of the processes' own rates (all cores busy).  Child processes
    are started fresh (spawn) and never touch the GPU."""
    import multiprocessing as mp
    import wmc_synth
    try:
        cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        cores = os.cpu_count() or 1
    procs = max(1, min(max_procs, cores))
    sizes = wmc_synth.c3_sizes()[:procs]
    jobs = [(b, h, w, s, iters) for b, (h, w, s) in enumerate(sizes)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_job, jobs)
    wall = time.perf_counter() - t0
    rate = sum(r[0] / r[1] for r in res)
    slowest = max(r[1] for r in res)
    return {"value": round(rate / 1e9, 6), "unit": "Gpixel-iter/s", "cores": procs,
            "sample": f"{procs} processes, one C3 image channel each, {iters} iterations "
                      f"(slowest {slowest:.1f} s, wall incl. start-up {wall:.1f} s)"}


def train_step_fn(torch, wmc, wmc_synth, dev, ckpt_every=5):
    """One optimisation step's worth of work on the 16 x 512 x 512, K = 20
    workload: the fused forward with checkpoints (every ceil(sqrt(K)) = 5
    steps unless given), the MSE loss against the clean images, and backward
    through the adjoint to f and lam."""
    noisy, clean = wmc_synth.c4()
    x = torch.from_numpy(noisy[:, 0]).to(dev)
    y = torch.from_numpy(clean[:, 0]).to(dev)
    lam16 = torch.ones(16, device=dev, requires_grad=True)
    xg = x.clone().requires_grad_(True)

    def step():
        # gradients cleared as an optimiser's zero_grad(set_to_none=True) does,
        # so autograd stores the new ones instead of adding them to the last
        xg.grad = None
        lam16.grad = None
        u = wmc.WMCSolve.apply(xg, lam16, 20, 0.0, ckpt_every)
        loss = torch.nn.functional.mse_loss(u, y)   # mean((u - y)^2), fused by torch
        loss.backward()
    return step, x


def timed(fn, reps, stream, torch):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


_SPIN = {"cycles_per_ms": None}


def timed_device(fn, reps, stream, torch, host_ms_per_call=0.5):
    """Device time of `reps` back-to-back calls of `fn`, with the host cost of
    issuing them hidden: a bounded spin kernel holds the stream while the host
    enqueues the calls, and the events bracket only the calls.  Returns
    (ms, hidden) where `hidden` says whether the enqueue finished before the
    spin did (else the figure still includes host time)."""
    if _SPIN["cycles_per_ms"] is None:
        cyc = 2_000_000
        torch.cuda._sleep(cyc)
        ms = timed(lambda: torch.cuda._sleep(cyc), 3, stream, torch) / 3
        _SPIN["cycles_per_ms"] = cyc / ms
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    es = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    spin_ms = 5.0 + host_ms_per_call * reps
    es.record(stream)
    torch.cuda._sleep(int(spin_ms * _SPIN["cycles_per_ms"]))
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    host_ms = (time.perf_counter() - t0) * 1e3
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1), host_ms < es.elapsed_time(e0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # defaults: 50 timed solves after 20 untimed ones; 10 after 3 read about
    # 1 % lower, the clocks still rising
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--side", type=int, default=4096)
    ap.add_argument("--no-extras", action="store_true", help="skip the step/batched extras")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=12,
                    help="iterations of the 4096^2 solve the CPU oracle runs (about 10 s)")
    ap.add_argument("--tuning", default="",
                    help="force the launch shape 'cols,tsteps,seg_rows' (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration for rocprofv3)")
    ap.add_argument("--only-extras", default="", metavar="NAMES",
                    help="run only these comma-separated extras and print them (profiling "
                         "runs; no main metric)")
    ap.add_argument("--train-only", type=int, default=0, metavar="N",
                    help="only run N training steps of the differentiable 16 x 512^2, K = 20 "
                         "solve (profiling runs)")
    ap.add_argument("--train-ckpt", type=int, default=5, metavar="C",
                    help="checkpoint period of --train-only (1: every state kept)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(sharding by image or by row band is a design only); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import wmc_synth
    import paper_1903_07189_amd as wmc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_dispatch": a.numel() * 4,
                          "copy_bytes_written_per_dispatch": a.numel() * 4}))
        return

    wmc.selftest()
    if args.train_only:
        step, _ = train_step_fn(torch, wmc, wmc_synth, dev, args.train_ckpt)
        step()
        ms = timed(step, args.train_only, stream, torch) / args.train_only
        print(json.dumps({"workload": "16 x 512^2 K=20 training step", "ckpt_every": args.train_ckpt,
                          "ms": round(ms, 4)}))
        return
    side, iters = args.side, args.iters
    noisy, _ = wmc_synth.c2(side=side)
    f = torch.from_numpy(noisy).to(dev)           # (1, side, side)
    lam = torch.tensor([1.0], device=dev)
    if args.only_extras:
        only = set(args.only_extras.split(","))
        unknown = only - set(EXTRA_NAMES)
        if unknown:
            sys.exit(f"unknown extras {sorted(unknown)}; known: {', '.join(EXTRA_NAMES)}")
        print(json.dumps(extras(torch, wmc, wmc_synth, f, lam, stream, side, only)), flush=True)
        return

    if args.tuning:
        c_, t_, r_ = (int(v) for v in args.tuning.split(","))
        tuning = {"cols": c_, "tsteps": t_, "seg_rows": r_, "use_graph": 1}
    else:
        tuning = wmc.solve_tuning(f, lam)         # autotuned once (cached) before timing
    plan = wmc.SolvePlan(f, lam, iters, tuning=tuning)
    for _ in range(args.warmup):
        plan()
    torch.cuda.synchronize()

    ms = timed(plan, args.steps, stream, torch)
    ms_per_step = ms / args.steps
    px_iter = side * side * iters
    value = px_iter / (ms_per_step * 1e-3) / 1e9

    launches = depths(iters, tuning["tsteps"])
    avg_launch_ms = ms_per_step / len(launches)
    mean_T = iters / len(launches)
    # dominant kernel: the fused streaming kernel; both of its bounds
    alu_achieved = ALGO_OPS_PER_PX_ITER * side * side * mean_T / (avg_launch_ms * 1e-3) / 1e12
    hbm_achieved = BYTES_PER_PX_PASS * side * side / (avg_launch_ms * 1e-3) / 1e9
    traffic = read_traffic(tuning, side)
    roof_alu = {"bound": "alu", "achieved": round(alu_achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "Tops/s", "frac": round(alu_achieved / ALU_PEAK_TOPS, 4), "traffic": traffic}
    roof_hbm = {"bound": "hbm", "achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    roofline = roof_alu if roof_alu["frac"] >= roof_hbm["frac"] else roof_hbm
    other = roof_hbm if roofline is roof_alu else roof_alu

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gpixel-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain WMC denoising solve, {side}x{side} fp32 piecewise-smooth "
                               f"synthetic + Gaussian noise sigma 0.1 (seed 1), {iters} iterations, "
                               "lam 1, dt 1/(1+lam)",
                   "side": side, "iters": iters, "lam": 1.0, "tuning": tuning,
                   "launches_per_step": len(launches), "kernel": "k_stream_single (fused, "
                   f"{tuning['tsteps']} sweeps/launch)"},
        "roofline": roofline,
        "roofline_other_bound": other,
        "traffic_note": "roofline.traffic = FETCH_SIZE + WRITE_SIZE per launch (rocprofv3, scaled "
                        "by a 1 GiB copy): traffic leaving the L2, Infinity Cache hits included "
                        "(the 192 MiB working set fits the 256 MB cache); extras.step_T1_8192 "
                        "is the update beyond the cache, against the probe of the same run",
        "step_equivalent_hbm_frac": round(BYTES_PER_PX_PASS * value / HBM_PEAK_GBS, 4),
        "paper_context": "33.2 Gpixel/s for the operator alone on an NVIDIA TITAN X (Pascal), "
                         "workload unstated (context only)",
    }

    if not args.no_extras:
        out["extras"] = extras(torch, wmc, wmc_synth, f, lam, stream, side)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(side, args.cpu_iters)
    print(json.dumps(out), flush=True)


EXTRA_NAMES = ("copy_ceiling", "step_T1_4096", "step_T1_8192", "compute_4096", "fd_4096", "l1_4096",
               "step_T1_4096_cold", "c4_train_step", "volume_256cubed", "layer_k8_16x512",
               "batched_c3", "c1_256", "c5_train_step")


def extras(torch, wmc, wmc_synth, f, lam, stream, side, only=None):
    ex = {}

    def want(name):
        return only is None or name in only
    if want("copy_ceiling"):
        ex.update(_copy_ceiling(torch, wmc, f, stream))
    if want("step_T1_4096") or want("step_T1_8192"):
        ex.update(_steps_t1(torch, wmc, f, lam, stream, side, want, ex))
    if want("compute_4096"):
        ms, hid = timed_device(lambda: wmc.compute(f), 20, stream, torch)
        ms /= 20
        ex["compute_4096"] = {"gpx_per_s": round(side * side / (ms * 1e-3) / 1e9, 1),
                              "gbs": round(8 * side * side / (ms * 1e-3) / 1e9, 1),
                              "host_hidden": hid}
    if want("fd_4096"):
        # conventional finite-difference comparator on the same image (8 B/px)
        ms, hid = timed_device(lambda: wmc.fd_compute(f), 20, stream, torch)
        ms /= 20
        ex["fd_4096"] = {"gpx_per_s": round(side * side / (ms * 1e-3) / 1e9, 1),
                         "gbs": round(8 * side * side / (ms * 1e-3) / 1e9, 1),
                         "host_hidden": hid}
    if want("l1_4096"):
        # l1-fidelity primal-dual solve on the same image, autotuned (20 B/px
        # per launch: U, d, f in; U, d out)
        wmc.solve_l1(f, 10.0, 0.05, 200)
        ms = timed(lambda: wmc.solve_l1(f, 10.0, 0.05, 200), 3, stream, torch) / 3
        ex["l1_4096"] = {"gpx_iter_s": round(side * side * 200 / (ms * 1e-3) / 1e9, 1),
                         "ms": round(ms, 3), "lam": 10.0, "alpha": 0.05, "iters": 200,
                         "note": "l1-fidelity primal-dual iteration, fused sweeps"}
    if want("step_T1_4096_cold"):
        ex.update(_step_cold(torch, f, lam, stream, side))
    if want("c4_train_step"):
        ex.update(_train(torch, wmc, wmc_synth, f, stream))
    if want("volume_256cubed"):
        ex.update(_volume(torch, wmc, f, stream))
    if want("layer_k8_16x512"):
        ex.update(_layer(torch, wmc, wmc_synth, f, stream))
    if want("c1_256"):
        # the 256 x 256 parity workload (seed 0, sigma 0.05, lam 1, 50
        # iterations): one graph-replayed solve, autotuned
        c1, _ = wmc_synth.c1()
        g1 = torch.from_numpy(c1).to(f.device)
        p1 = wmc.SolvePlan(g1, lam, 50, tuning=wmc.solve_tuning(g1, lam))
        p1()
        ms = timed(p1, 50, stream, torch) / 50
        ex["c1_256"] = {"ms_per_solve": round(ms, 4),
                        "gpx_iter_s": round(256 * 256 * 50 / (ms * 1e-3) / 1e9, 2),
                        "note": "256x256 fp32, 50 iterations, one graph replay per solve"}
        del g1
    if want("c5_train_step"):
        # one optimiser step of the learned-lambda workload: 32 x 256^2
        # (seed 3000), lambda from an 8-entry table, K = 30, a checkpoint
        # every ceil(sqrt(K)) = 6 steps, MSE loss, backward to the table
        noisy, clean, _ = wmc_synth.c5_batch(3000, batch=32)
        x5 = torch.from_numpy(noisy[:, 0]).to(f.device)
        y5 = torch.from_numpy(clean[:, 0]).to(f.device)
        theta = torch.zeros(8, device=f.device, requires_grad=True)
        k5 = torch.arange(32, device=f.device) % 8

        def step5():
            u = wmc.WMCSolve.apply(x5, torch.exp(theta)[k5], 30, 0.0, 6)
            torch.nn.functional.mse_loss(u, y5).backward()
        for _ in range(3):
            step5()
        ms = timed(step5, 20, stream, torch) / 20
        ms_d, hid = timed_device(step5, 20, stream, torch, host_ms_per_call=3.0)
        ex["c5_train_step"] = {"ms": round(ms, 3), "ms_device": round(ms_d / 20, 3),
                               "host_hidden": hid,
                               "ckpt_every": 6,
                               "note": "32x256^2, K=30, forward + MSE + backward to the lambda table"}
        del x5, y5
    if want("batched_c3"):
        ex.update(_batched(torch, wmc, wmc_synth, f, stream))
    return ex


def probe_ceiling(torch, wmc, side, stream, reps=20):
    """Achievable streaming bandwidth (GB/s) from the library's probe kernel
    (wmc_bw_probe) over side^2 fp32 planes: copy (one read, one write) and
    add o = a + b (two reads, one write: the single update's pattern), with
    plain and with non-temporal accesses."""
    n = side * side
    a = torch.rand(n, device="cuda:0")
    b = torch.rand_like(a)
    o = torch.empty_like(a)
    out = {}
    for op in ("copy", "add"):
        for nt in (False, True):
            def run():
                wmc.bw_probe(a, o, b if op == "add" else None, nontemporal=nt)
            run()
            ms = timed(run, reps, stream, torch) / reps
            planes = 3 if op == "add" else 2
            out[f"{op}{'_nt' if nt else ''}"] = round(planes * n * 4 / (ms * 1e-3) / 1e9, 1)
    del a, b, o
    return out


def _copy_ceiling(torch, wmc, f, stream):
    ex = {}
    # the library's streaming probe: 8192^2 planes (256 MiB each; the add's
    # 768 MiB exceed the 256 MB Infinity Cache) and 4096^2 (cache-resident)
    p8 = probe_ceiling(torch, wmc, 8192, stream)
    p4 = probe_ceiling(torch, wmc, 4096, stream)
    ex["probe_8192"] = dict(p8, note="wmc_bw_probe GB/s: copy and o = a + b over 8192^2 fp32, "
                                     "plain and non-temporal")
    ex["probe_4096"] = dict(p4, note="the same over 4096^2 (working set inside the Infinity Cache)")
    return ex


def _steps_t1(torch, wmc, f, lam, stream, side, want, probes):
    ex = {}
    # plain single-update kernel (one launch per iteration, graph-replayed); the
    # launch shape is picked from a few candidates, best reported
    reps = 50

    def t1_gbs(img, side_, iters_, shapes):
        best = (0.0, None)
        for c_, r_ in shapes:
            t1 = {"cols": c_, "tsteps": 1, "seg_rows": r_, "use_graph": 1}
            p1 = wmc.SolvePlan(img, lam, iters_, tuning=t1)
            p1()
            ms = timed(p1, 3, stream, torch) / 3
            gbs = BYTES_PER_PX_PASS * side_ * side_ / (ms / iters_ * 1e-3) / 1e9
            if gbs > best[0]:
                best = (gbs, t1)
        return best

    if want("step_T1_4096"):
        gbs, t1 = t1_gbs(f, side, reps,
                         [(2, 14), (2, 16), (2, 28), (2, 32), (4, 8), (4, 23), (4, 32)])
        ex["step_T1_4096"] = {"gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                              "gpx_per_s": round(gbs / BYTES_PER_PX_PASS, 2), "tuning": t1,
                              "note": "warm: the 192 MiB working set fits the 256 MB Infinity "
                                      "Cache"}
        if "probe_4096" in probes:
            ex["step_T1_4096"]["probe_add_frac"] = round(gbs / probes["probe_4096"]["add"], 4)
    if want("step_T1_8192"):
        # 8192^2 control, larger than the Infinity Cache
        g = torch.rand((1, 8192, 8192), device=f.device)
        gbs, t1 = t1_gbs(g, 8192, 20, [(4, 2), (4, 3), (4, 4), (4, 8), (2, 4), (2, 14), (4, 12)])
        ex["step_T1_8192"] = {"gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                              "tuning": t1,
                              "note": "768 MiB working set, beyond the Infinity Cache"}
        if "probe_8192" in probes:
            p8 = probes["probe_8192"]
            ex["step_T1_8192"]["probe_add_frac"] = round(gbs / p8["add"], 4)
            ex["step_T1_8192"]["probe_add_nt_frac"] = round(gbs / p8["add_nt"], 4)
        del g
    return ex


def _step_cold(torch, f, lam, stream, side):
    ex = {}
    # cold single update: four independent 4096^2 problems (768 MiB, three
    # times the Infinity Cache) updated round-robin, so every launch finds its
    # operands evicted; wmc_step launches enqueued back to back through the ABI
    from paper_1903_07189_amd import wmc as M
    L = M.lib()
    us = [torch.rand_like(f) for _ in range(4)]
    fs = [torch.rand_like(f) for _ in range(4)]
    outs = [torch.empty_like(f) for _ in range(4)]
    shp, st = M.shape_of(f), M._stream()

    def run_cold():
        for i in range(4):
            M.check(L.wmc_step(M._ptr(us[i]), M._ptr(fs[i]), M._ptr(outs[i]), M._ptr(lam), 0.0,
                               None, shp, st))
    run_cold()
    ms = timed(run_cold, 10, stream, torch) / 40
    ex["step_T1_4096_cold"] = {"gbs": round(BYTES_PER_PX_PASS * side * side / (ms * 1e-3) / 1e9, 1),
                               "us_per_launch": round(ms * 1e3, 2),
                               "note": "wmc_step, 4 problems round-robin (768 MiB > Infinity Cache)"}
    del us, fs, outs
    return ex


def _train(torch, wmc, wmc_synth, f, stream):
    ex = {}
    # differentiable solve (16 x 512 x 512, K = 20, checkpoint every 5): one
    # training step = fused forward with checkpoints + hand-written adjoint
    pxs = 16 * 512 * 512 * 20
    lam16 = torch.ones(16, device=f.device)
    for name, c in (("c4_train_step", 5), ("c4_train_step_every_state", 1)):
        train_step, x = train_step_fn(torch, wmc, wmc_synth, f.device, c)
        for _ in range(3):   # warm-up: first-call set-up (tuning, plan caches) outside the timing
            train_step()
        ms_t = timed(train_step, 20, stream, torch) / 20
        # the same steps with the host's enqueueing hidden behind a spin
        # kernel: the device time of a step
        ms_d, hid = timed_device(train_step, 20, stream, torch, host_ms_per_call=3.0)
        ms_d /= 20
        cc = c or wmc.wmc.default_ckpt_every(20, x.numel() * 4)
        ms_f = timed(lambda: wmc.solve(x, lam16, 20, ckpt_every=cc), 20, stream, torch) / 20
        ex[name] = {"ckpt_every": cc, "ms_forward_backward": round(ms_t, 3),
                    "ms_forward_backward_device": round(ms_d, 3), "host_hidden": hid,
                    "ms_forward_ckpt": round(ms_f, 3),
                    "forward_gpx_iter_s": round(pxs / (ms_f * 1e-3) / 1e9, 1),
                    "backward_gpx_step_s": round(pxs / ((ms_t - ms_f) * 1e-3) / 1e9, 1),
                    "note": "c4_train_step checkpoints every ceil(sqrt(K)) = 5 steps; "
                            "c4_train_step_every_state keeps every state (period 1, the "
                            "library's default while K states fit 2 GiB); backward = segment "
                            "recompute (none at period 1) + adjoint steps + lam reduction"}
        del x
    return ex


def _volume(torch, wmc, f, stream):
    ex = {}
    # 3-D extension: one 256^3 volume, operator and data-term Jacobi steps
    vol = torch.rand((256, 256, 256), device=f.device)
    ms_c3, hid_c = timed_device(lambda: wmc.compute3(vol), 10, stream, torch)
    ms_s3, hid_s = timed_device(lambda: wmc.solve3(vol, 1.0, 10), 3, stream, torch)
    ms_c3 /= 10
    ms_s3 /= 3
    nv = vol.numel()
    # differentiable 3-D solve: K = 5 steps, one checkpoint (the backward
    # recomputes four states), adjoint = selection pass + gather per step
    K3 = 5
    lam3 = torch.ones(1, device=f.device)
    out3, ck3 = wmc.solve3(vol, lam3, K3, ckpt_every=K3)
    g3 = torch.rand_like(out3)
    ms_b3, hid_b = timed_device(lambda: wmc.backward3(g3, vol, lam3, K3, ck3, K3), 3, stream, torch)
    ms_b3 /= 3
    ex["volume_256cubed"] = {"compute_gvox_s": round(nv / (ms_c3 * 1e-3) / 1e9, 1),
                             "solve_gvox_iter_s": round(nv * 10 / (ms_s3 * 1e-3) / 1e9, 1),
                             "backward_ms_k5": round(ms_b3, 3),
                             "backward_gvox_step_s": round(nv * K3 / (ms_b3 * 1e-3) / 1e9, 1),
                             "host_hidden": hid_c and hid_s and hid_b,
                             "note": "18 half windows, one sweep per launch; backward of a "
                                     "5-step solve from one checkpoint (4 states recomputed)"}
    del vol, out3, ck3, g3
    return ex


def _layer(torch, wmc, wmc_synth, f, stream):
    ex = {}
    # learnable half-window layer, 8 kernels, on the 16 x 512^2 batch
    xw = torch.from_numpy(wmc_synth.c4()[0][:, 0]).to(f.device)
    kw = wmc.nn.printed_kernels(device=f.device)
    out_l, sel_l = wmc.layer_forward(xw, kw)
    gl = torch.randn_like(xw)
    reps = 20
    ms_lf, h1 = timed_device(lambda: wmc.layer_forward(xw, kw), reps, stream, torch)
    ms_lb, h2 = timed_device(lambda: wmc.layer_backward(xw, kw, sel_l, gl), reps, stream, torch)
    ms_lu, h3 = timed_device(lambda: wmc.layer_backward(xw, kw, sel_l, gl, need_w=False), reps,
                             stream, torch)
    ms_lf, ms_lb, ms_lu = ms_lf / reps, ms_lb / reps, ms_lu / reps
    npx = xw.numel()
    ex["layer_k8_16x512"] = {"forward_gpx_s": round(npx / (ms_lf * 1e-3) / 1e9, 1),
                             "backward_gpx_s": round(npx / (ms_lb * 1e-3) / 1e9, 1),
                             "backward_input_grad_only_gpx_s": round(npx / (ms_lu * 1e-3) / 1e9, 1),
                             "ms_forward": round(ms_lf, 4), "ms_backward": round(ms_lb, 4),
                             "host_hidden": h1 and h2 and h3}
    del xw, out_l, sel_l, gl
    return ex


def _batched(torch, wmc, wmc_synth, f, stream):
    ex = {}
    # uneven batch: 64 images x 3 channels, sides U{128..2048}, 100 iterations
    sizes = wmc_synth.c3_sizes()
    imgs = []
    for b, (hh, ww, sig) in enumerate(sizes):
        noisy, _ = wmc_synth.c3_image(b, hh, ww, sig)
        imgs.append(torch.from_numpy(noisy).to(f.device))
    lams = torch.ones(len(imgs), device=f.device)
    px = sum(int(x.numel()) for x in imgs)
    bp = wmc.SolveBatchedPlan(imgs, lams, 100)
    bp()  # autotunes once
    ms_b = timed(bp, 3, stream, torch) / 3
    # per-image plain form: per image one single-update launch per iteration, no graph
    plain = {"cols": 2, "tsteps": 1, "seg_rows": 32, "use_graph": 0}
    plans = [wmc.SolvePlan(x, lams[i:i + 1].expand(x.shape[0]).contiguous(), 100, tuning=plain)
             for i, x in enumerate(imgs)]

    def run_plain():
        for p in plans:
            p()
    run_plain()
    ms_p = timed(run_plain, 2, stream, torch) / 2
    # per image, graph-replayed fused solves (the library's best single-image path)
    gplans = [wmc.SolvePlan(x, lams[i:i + 1].expand(x.shape[0]).contiguous(), 100)
              for i, x in enumerate(imgs)]

    def run_graphed():
        for p in gplans:
            p()
    run_graphed()
    ms_g = timed(run_graphed, 2, stream, torch) / 2
    ex["batched_c3"] = {"channel_px": px, "iters": 100,
                        "per_image_graphed_gpx_iter_s": round(px * 100 / (ms_g * 1e-3) / 1e9, 2),
                        "speedup_vs_graphed": round(ms_g / ms_b, 2),
                        "batched_gpx_iter_s": round(px * 100 / (ms_b * 1e-3) / 1e9, 2),
                        "per_image_plain_gpx_iter_s": round(px * 100 / (ms_p * 1e-3) / 1e9, 2),
                        "speedup": round(ms_p / ms_b, 2), "ms_batched": round(ms_b, 3),
                        "ms_per_image_plain": round(ms_p, 3),
                        "per_image_plain_launches": 100 * len(imgs)}
    return ex


if __name__ == "__main__":
    main()
