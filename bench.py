"""Benchmark: batched complex FFT throughput on one MI355X.

A step is one pass of the batched-FFT hot path over the headline workload:
complex64 transforms of N = 256, 1024 and 4096, each at batch 2^24 / N
(2^24 elements, 256 MiB of algorithmic HBM traffic per launch), forward and
inverse -- six launches per step.  Inputs are seeded uniform[-1, 1) and
resident in HBM before timing; four input/output buffer pairs (1 GiB) rotate
so the 256 MB last-level cache does not serve the reads.

Prints one JSON line.  `value` is GFLOP/s in the 5 N log2 N convention.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SIZES = (256, 1024, 4096)
ELEMS = 1 << 24
NBUF = 4


def flops(n, batch):
    return 5.0 * n * math.log2(n) * batch if n > 1 else 0.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--extras", default="c128",
                    help="comma list of extra measurements: c128 (default), none")
    return ap.parse_args()


class KernelTimer:
    """Average duration of repeated launches of one plan, timed with HIP events
    recorded on the stream the kernels run on."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, plan, xs, ys, reps):
        torch = self.torch
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for i in range(3):
            plan.execute(xs[i % len(xs)], ys[i % len(ys)], s)
        e0.record(s)
        for i in range(reps):
            plan.execute(xs[i % len(xs)], ys[i % len(ys)], s)
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps  # ms


def cpu_baseline(seconds):
    """The FP64 O(N^2) oracle on the host cores, on a bounded sample of the
    same workload (transforms of each N, both directions)."""
    import oracle
    from paper_2207_06803_amd import synth
    threads = oracle.max_threads()
    g = synth.rng(1, 77)
    # calibrate: one transform per size
    per = {}
    for n in SIZES:
        x = synth.uniform_complex(g, (threads, n), np.complex64)
        t0 = time.perf_counter()
        oracle.dft(x, -1)
        per[n] = (time.perf_counter() - t0) / threads
    budget = seconds / (2 * len(SIZES))
    tot_flops, tot_t, counts = 0.0, 0.0, {}
    for n in SIZES:
        cnt = max(threads, int(budget / per[n]) // threads * threads)
        counts[n] = cnt
        x = synth.uniform_complex(g, (cnt, n), np.complex64)
        for sign in (-1, 1):
            t0 = time.perf_counter()
            oracle.dft(x, sign)
            tot_t += time.perf_counter() - t0
            tot_flops += flops(n, cnt)
    return {"value": tot_flops / tot_t / 1e9, "unit": "GFLOP/s (5 N log2 N)", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 O(N^2) oracle, complex64 inputs, forward+inverse, transforms per N: "
                      + ", ".join(f"{n}:{c}" for n, c in counts.items()),
            "seconds": tot_t}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_2207_06803_amd import fftc, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # seeded inputs, generated once on the host and copied to HBM
    g = synth.rng(1, 0)
    host = synth.uniform_complex(g, (ELEMS,), np.complex64)
    xs = [torch.from_numpy(host).to(dev) for _ in range(NBUF)]
    for i in range(1, NBUF):
        xs[i].mul_(1.0 + 0.0625 * i)
    ys = [torch.empty_like(xs[0]) for _ in range(NBUF)]

    plans = []
    for n in SIZES:
        for d in (fftc.FORWARD, fftc.INVERSE):
            plans.append(fftc.Plan(n, ELEMS // n, d, "c64"))
    step_flops = sum(flops(p.n, p.batch) for p in plans)
    step_bytes = sum(16.0 * p.n * p.batch for p in plans)
    s = torch.cuda.current_stream()

    def step(i):
        for j, p in enumerate(plans):
            k = (i * len(plans) + j) % NBUF
            p.execute(xs[k], ys[k], s)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall0 = time.perf_counter()
    e0.record(s)
    for i in range(args.steps):
        step(i)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    value = step_flops / (ms_step * 1e-3) / 1e9

    # per-kernel average durations (HIP events on the launch stream)
    kt = KernelTimer(torch)
    per = {}
    for p in plans:
        avg = kt.time(p, xs, ys, 20)
        per[f"{p.n}_{'fwd' if p.direction < 0 else 'inv'}"] = {
            "ms": avg, "gflops": flops(p.n, p.batch) / (avg * 1e-3) / 1e9,
            "hbm_gbs": 16.0 * p.n * p.batch / (avg * 1e-3) / 1e9,
            "radices": p.describe()["radices"], "variant": p.describe()["variant"]}
    dom_key = max(per, key=lambda k: per[k]["ms"])
    dom = per[dom_key]
    roofline = {"bound": "hbm", "kernel": f"stockham c64 N={dom_key}", "achieved": dom["hbm_gbs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["hbm_gbs"] / HBM_PEAK_GBS,
                "traffic": None}

    extras = {}
    if "c128" in args.extras:
        xs128 = [torch.from_numpy(synth.uniform_complex(synth.rng(1, 1), (ELEMS,), np.complex128)).to(dev)
                 for _ in range(2)]
        ys128 = [torch.empty_like(xs128[0]) for _ in range(2)]
        for n in SIZES:
            for d in (fftc.FORWARD, fftc.INVERSE):
                with fftc.Plan(n, ELEMS // n, d, "c128") as p:
                    avg = kt.time(p, xs128, ys128, 10)
                extras[f"c128_{n}_{'fwd' if d < 0 else 'inv'}"] = {
                    "ms": avg, "gflops": flops(n, ELEMS // n) / (avg * 1e-3) / 1e9,
                    "hbm_gbs": 32.0 * ELEMS / (avg * 1e-3) / 1e9}
        del xs128, ys128

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)

    out = {
        "metric": "complex64 FFT GFLOP/s (5Nlog2N) & HBM GB/s; served p50/p99 latency",
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 arithmetic)",
        "data": "synthetic: seeded uniform[-1,1) re/im",
        "config": {"workload": "batched complex64 FFT, N in {256,1024,4096}, batch 2^24/N, "
                               "forward+inverse (6 launches per step)",
                   "elements_per_launch": ELEMS, "rotating_buffers": NBUF},
        "hbm_gbs": step_bytes / (ms_step * 1e-3) / 1e9,
        "wall_s": wall,
        "per_kernel": per,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    for p in plans:
        p.close()


if __name__ == "__main__":
    main()
