#!/usr/bin/env python3
"""Throughput benchmark: picoseconds per attempted spin flip on one MI355X.

A step is one complete run of the mid-size workload through the C-ABI
library: regenerate the couplings and initial spins on the device, then
10^5 red/black Metropolis sweeps of an L = 64 sample with two replicas
(p = 0.5, T = 0.7), snapshots at t_w in {10^2, 10^3, 10^4} and 20
log-spaced measurements of energy, magnetisation, overlap, C(t, t_w) and
C4(r).  ps/flip = step time / (sweeps x L^3 x 2 replicas).

Printed as one JSON line, with
  roofline      the half-step kernel's achieved integer-ALU rate (algorithmic
                lane-ops per launch over its event-timed average duration)
                against the chip's peak;
  cpu_baseline  the CPU oracle timed on a bounded sample of the same run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ps per spin flip (batched vs plain, 1 MI355X, bit-exact); HBM/VALU % of peak"

# Integer-ALU roofline.  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz simple
# 32-bit lane-ops per second.  Algorithmic work per attempted flip: a quarter
# of a Philox4x32-10 block (10 rounds x (2 multiply-hi-lo + 2 three-way XOR)
# = 40 lane-ops per 4 words) plus one compare of the word with the threshold.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
ALG_OPS_PER_FLIP = 40 / 4 + 1


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def run_job(sim, job):
    """One full run of the job on an already allocated sim (synchronous)."""
    sim.reset(job.seed, job.sample)
    t = 0
    for te, slots, meas in job.events():
        if te > t:
            sim.sweep(te - t)
            t = te
        for k in slots:
            sim.snapshot(k)
        if meas:
            sim.measure()
    if job.n_sweeps > t:
        sim.sweep(job.n_sweeps - t)
    sim.sync()


def cpu_baseline(job, sweeps: int):
    import oracle
    oracle.build()
    o = oracle.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
    t0 = time.perf_counter()
    o.sweep(sweeps)
    dt = time.perf_counter() - t0
    flips = sweeps * 2 * job.L ** 3
    return {"value": dt / flips * 1e12, "unit": "ps/flip", "cores": 1, "kind": "oracle",
            "sample": f"L={job.L} p={job.p} T={job.T} seed={job.seed}: the first {sweeps} sweeps "
                      f"of the run ({flips} attempted flips, {dt:.1f} s, single thread)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=100_000, help="sweeps per run (step)")
    ap.add_argument("--burst", type=int, default=2048, help="sweeps in the kernel-timing burst")
    ap.add_argument("--cpu-sweeps", type=int, default=60, help="oracle sweeps for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); every job is "
              "independent, so more GPUs would shard jobs without any exchange.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1411_5512_amd as ea
    from paper_1411_5512_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    job = wl.mid_job(args.sweeps)
    sim = ea.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
    stream = sim.stream
    flips_per_step = job.flips

    for i in range(args.warmup):
        run_job(sim, job)
        log(f"warmup {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    w0 = time.perf_counter()
    for i in range(args.steps):
        run_job(sim, job)
        log(f"step {i + 1}/{args.steps} done")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    dev_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / args.steps
    ps_per_flip = ms_per_step * 1e-3 / flips_per_step * 1e12

    # Sweeps only (no measurement or reset), for the roofline: a burst of
    # half-step launches timed with events on the run's stream.
    sim.reset(job.seed, job.sample)
    sim.sweep(64)
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    sim.sweep(args.burst)
    b1.record(stream)
    torch.cuda.synchronize()
    burst_ms = b0.elapsed_time(b1)
    launches = 2 * args.burst
    avg_launch_s = burst_ms * 1e-3 / launches
    flips_per_launch = job.L ** 3  # N/2 sites in each of the two replicas
    achieved = ALG_OPS_PER_FLIP * flips_per_launch / avg_launch_s / 1e12
    sweeps_only_ps = burst_ms * 1e-3 / (args.burst * 2 * job.L ** 3) * 1e12
    log(f"step {ms_per_step:.1f} ms ({ps_per_flip:.3f} ps/flip); half-step avg {avg_launch_s * 1e6:.2f} us")

    out = {
        "metric": METRIC,
        "value": round(ps_per_flip, 4),
        "unit": "ps/flip",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"plain form, mid size: L={job.L}, p={job.p}, T={job.T}, 1 sample x 2 replicas, "
                        f"{job.n_sweeps} sweeps, {len(job.meas_t)} measurements, tw={job.tw}",
            "form": "plain (one launch per half-step, sweeps replayed from a captured graph)",
            "L": job.L, "p": job.p, "T": job.T, "sweeps": job.n_sweeps,
            "flips_per_step": flips_per_step,
        },
        "device_ms_per_step": round(dev_ms / args.steps, 3),
        "sweeps_only_ps_per_flip": round(sweeps_only_ps, 4),
        "roofline": {
            "bound": "alu",
            "kernel": "half_step_kernel<32>",
            "achieved": round(achieved, 4),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s (32-bit lane-ops)",
            "frac": round(achieved / VALU_PEAK_TOPS, 5),
            "traffic": None,
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "alg_ops_per_flip": ALG_OPS_PER_FLIP,
            "flips_per_launch": flips_per_launch,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(job, args.cpu_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
