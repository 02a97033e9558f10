#!/usr/bin/env python3
"""Throughput benchmark: picoseconds per attempted spin flip on one MI355X,
batched form against the plain form.

Batched workload (the timed step): 256 independent disorder samples with two
replicas each, L drawn from {24, 32, 48, 64}, p from {0.5, 0.3, 0.2}, T from
{0.6, 0.8, 1.0} (seeds 0..255), 10^5 red/black Metropolis sweeps each with 20
log-spaced measurements of energy, magnetisation, overlap, C(t, t_w), C4(r)
and snapshots at t_w in {10^2, 10^3, 10^4}.  A step regenerates every job's
couplings and initial spins on the device and runs all jobs to the end in
one persistent launch; the two are captured as one hipGraph and replayed.
ps/flip = step time / sum_jobs(sweeps x L^3 x 2).

Plain workload (reported beside it): one L = 64 sample, p = 0.5, T = 0.7,
the same schedule shape, one kernel launch per half-step.

One JSON line is printed, with
  roofline      the dominant kernel's achieved integer-ALU rate (algorithmic
                lane-ops per launch over its event-timed duration) against the
                chip's peak;
  cpu_baseline  the CPU oracle timed on a bounded sample of the plain run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# The serving leg drives its streamed jobs from four workers, each with its own
# stream, beside the batched launch's stream; HIP maps streams onto the
# process's hardware queues in turn (4 by default), and persistent launches
# that share a queue run one after the other.  Eight queues let all five run
# at once; set before anything initialises HIP (the library reads the same
# variable to size its workers).
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ps per spin flip (batched vs plain, 1 MI355X, bit-exact); HBM/VALU % of peak"

# Integer-ALU roofline.  Peak: the chip's vector lane rate, 256 CUs x 4 SIMDs
# x 32 lanes x 2.4 GHz = 78.6e12 lane-ops/s (the fp32 vector peak of
# 157.3 TFLOP/s counts an FMA as two flops in one lane slot).  Algorithmic
# work per attempted flip in those slots: a quarter of a Philox4x32-10 block
# (10 rounds x (2 multiply-hi-lo + 2 three-way XOR) per 4 words), where a
# 32x32->64-bit multiply-add takes two slots (the --alu-probe measures
# v_mad_u64_u32 at half the rate of v_bitop3_b32), plus one compare of the
# word with its threshold: 5 x 2 + 5 + 1 = 16.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
ALG_OPS_PER_FLIP = 16.0

# HBM bytes per launch of the batched kernel on this workload, measured with
# rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by a device-to-device copy of
# known size) and recorded with a hash of the kernel sources they were taken
# on; reported only while the sources still hash the same.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_kernel_mixed256_traffic.txt")
KERNEL_SOURCES = ("ea_device.h", "ea_kernels.h", "ea_batch_kernels.h", "ea_batch_api.h")
# the same for the multispin half-step on the paper's production batch
MSC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "msc_half_step_L128_B64_traffic.txt")
MSC_SOURCES = ("ea_device.h", "ea_msc_kernels.h", "ea_msc_api.h")


def kernel_source_hash(sources=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in sources or KERNEL_SOURCES:
        h.update(name.encode() + b"\0")
        with open(os.path.join(ROOT, "paper_1411_5512_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_record(path=None, sources=None):
    """The recorded counters (dict) if they were taken on the current kernel
    sources, else (None, reason).  Defaults: the batched kernel's record."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            kv = dict(line.split(None, 1) for line in f if line.strip() and not line.startswith("#"))
    except OSError:
        return None, "no counter record"
    kv = {k: v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash(sources):
        return None, "kernel changed since the counters were taken"
    return kv, kv.get("workload", "")


def measured_traffic(path=None, sources=None):
    """(HBM bytes per launch, provenance) from the record, or (None, reason)."""
    kv, why = measured_record(path, sources)
    if kv is None:
        return None, why
    return int(kv["fetch_bytes"]) + int(kv["write_bytes"]), why


def algorithmic_bytes(jobs) -> int:
    """State traffic the batched form cannot avoid, packed bits: per replica
    the spins and couplings loaded once and the spins stored once; per
    snapshot the replica written; per measurement each replica published and
    read back for the pair observables, and each taken snapshot read."""
    total = 0
    for j in jobs:
        rep = j.L ** 3 // 8  # bytes of one replica's spins
        total += 2 * (rep + 3 * rep + rep) + 2 * rep * len(j.tw)
        for t in j.meas_t:
            taken = sum(1 for w in j.tw if w <= t)
            total += 2 * (rep + rep + taken * rep)
    return total


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def run_plain_job(sim, job):
    """One full plain run on an already allocated sim (synchronous)."""
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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(job, sweeps: int, agg_procs: int, agg_sweeps: int):
    """The oracle on the host: one thread on the first `sweeps` sweeps of the
    job, then `agg_procs` independent processes (one sample each, seeds
    1..agg_procs) running `agg_sweeps` sweeps at once for an all-core rate."""
    import subprocess
    import oracle
    oracle.build()
    o = oracle.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
    t0 = time.perf_counter()
    o.sweep(sweeps)
    dt = time.perf_counter() - t0
    flips = sweeps * 2 * job.L ** 3
    out = {"value": round(dt / flips * 1e12, 1), "unit": "ps/flip", "cores": 1, "kind": "oracle",
           "cpu": _cpu_model(),
           "sample": f"plain run L={job.L} p={job.p} T={job.T} seed={job.seed}: its first {sweeps} sweeps "
                     f"({flips} attempted flips, {dt:.1f} s, one thread)"}
    if agg_procs > 0 and agg_sweeps > 0:
        code = ("import sys, time; sys.path.insert(0, sys.argv[1]); import oracle; "
                "o = oracle.Sim(int(sys.argv[2]), float(sys.argv[3]), float(sys.argv[4]), seed=int(sys.argv[5])); "
                "t = time.perf_counter(); o.sweep(int(sys.argv[6])); print(time.perf_counter() - t)")
        procs = [subprocess.Popen([sys.executable, "-c", code, ROOT, str(job.L), str(job.p), str(job.T),
                                   str(1 + i), str(agg_sweeps)], stdout=subprocess.PIPE, text=True)
                 for i in range(agg_procs)]
        times = [float(p.communicate(timeout=600)[0].strip().splitlines()[-1]) for p in procs]
        agg_flips = agg_procs * agg_sweeps * 2 * job.L ** 3
        out["all_cores"] = {"value": round(max(times) / agg_flips * 1e12, 2), "unit": "ps/flip",
                            "cores": agg_procs,
                            "sample": f"{agg_procs} processes at once, one sample each (seeds 1..{agg_procs}), "
                                      f"{agg_sweeps} sweeps of L={job.L}; slowest process {max(times):.1f} s"}
    return out


def bench_plain(ea, torch, job, steps: int, burst: int):
    tuned = ea.tune_plain(job.L)  # untimed: picks the bit packing of the plain form for this size
    sim = ea.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
    stream = sim.stream
    run_plain_job(sim, job)  # warm-up
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(steps):
        run_plain_job(sim, job)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - w0) * 1e3 / steps
    # one slab launch of `burst` sweeps timed with events on the run's stream
    sim.reset(job.seed, job.sample)
    sim.sweep(64)
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    sim.sweep(burst)
    b1.record(stream)
    torch.cuda.synchronize()
    sweep_us = b0.elapsed_time(b1) * 1e3 / burst
    plan = sim.slab_plan
    sim.close()
    alu = ALG_OPS_PER_FLIP * 2 * job.L ** 3 / (sweep_us * 1e-6) / 1e12
    # the latency that bounds one-plane slabs: every half-step waits for one
    # exchange with the neighbouring slabs, whose chain crosses XCDs
    xchg = exchange_probe()
    floor_us = 2 * xchg.get("one_way_us_other_xcd", xchg.get("one_way_us_same_xcd", 0.0))
    return {
        "workload": f"L={job.L} p={job.p} T={job.T}, 1 sample x 2 replicas, {job.n_sweeps} sweeps, "
                    f"{len(job.meas_t)} measurements, tw={job.tw}; persistent slab launches between events",
        "words_per_row": tuned["words_per_row"],
        "slab_plan": {"slabs_per_replica": plan[0], "ghost_planes": plan[1]},
        "ps_per_flip": round(ms * 1e-3 / job.flips * 1e12, 4),
        "ms_per_step": round(ms, 3),
        "steps": steps,
        "sweep_avg_us": round(sweep_us, 3),
        "ps_per_flip_sweeps": round(sweep_us * 1e-6 / (2 * job.L ** 3) * 1e12, 4),
        "alu_frac": round(alu / VALU_PEAK_TOPS, 5),
        "latency_floor": {"bound": "exchange latency", "exchange": xchg,
                          "floor_us_per_sweep": round(floor_us, 3),
                          "note": "two one-way exchanges per sweep (one per half-step), measured live; the "
                                  "update of a slab's words adds one dependent chain per half-step",
                          "frac": round(floor_us / sweep_us, 4) if sweep_us > 0 else None},
    }


def alu_probe():
    """Sustained lane rate of the instructions the roofline counts as one
    lane-op each (libea_probe.so, event-timed launches of 4 waves per SIMD
    on every CU): v_mad_u64_u32, v_bitop3_b32, and whole Philox4x32-10
    blocks at 40 lane-ops each."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1411_5512_amd", "libea_probe.so"))
    lib.ea_probe_alu.restype = ctypes.c_int
    lib.ea_probe_alu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
    out = {"peak_tops": round(VALU_PEAK_TOPS, 2), "threads_per_block": 256,
           "note": "blocks = 256 CUs x 16 (many waves per SIMD) or 256 CUs x 4 (four per SIMD, as the update "
                   "kernels run); philox counts 40 lane-ops per block (the roofline's count, in which a "
                   "multiply-add is one op)"}
    probes = ((0, "v_mad_u64_u32", 20000), (1, "v_bitop3_b32", 20000), (3, "philox_1_chain", 4000),
              (2, "philox_2_chains", 4000), (4, "philox_4_chains", 2000))
    for blocks in (256 * 16, 256 * 4):
        for kind, name, iters in probes:
            ms, ops = ctypes.c_double(0.0), ctypes.c_double(0.0)
            rc = lib.ea_probe_alu(kind, blocks, iters * 16 * 256 // blocks, ctypes.byref(ms), ctypes.byref(ops))
            if rc != 0:
                raise RuntimeError(f"ea_probe_alu({name}) failed: {rc}")
            tops = ops.value / (ms.value * 1e-3) / 1e12
            out[f"{name}@{blocks // 256}wg_per_cu"] = {"ms": round(ms.value, 3), "lane_ops": ops.value,
                                                       "tops": round(tops, 3),
                                                       "frac_of_peak": round(tops / VALU_PEAK_TOPS, 4)}
    return out


def shells_probe(ea, sizes=(32, 64, 128, 256), reps=3, direct_sizes=(32, 64, 128, 256)):
    """Wall time of one full-vector C4 call (ea_c4_shells over every
    displacement, synchronous) by the FFT route, and by the direct route at
    `direct_sizes`, on a quenched run of each size after 20 sweeps; where both
    run, the results must be identical.  The first call of each route
    allocates its scratch, so the best of `reps` later calls is reported."""
    out = {}
    try:
        for L in sizes:
            g = ea.Sim(L, 0.5, 0.7, seed=1)
            g.sweep(20)
            n_all = 3 * (L // 2) ** 2 + 1
            row, res = {}, {}
            routes = [("fft", ea.SHELLS_FFT)] + ([("direct", ea.SHELLS_DIRECT)] if L in direct_sizes else [])
            for name, route in routes:
                ea.set_shell_route(route)
                res[name] = g.c4_shells(n_all)
                best = float("inf")
                for _ in range(reps if name == "fft" or L <= 128 else 1):
                    t0 = time.perf_counter()
                    g.c4_shells(n_all)
                    best = min(best, time.perf_counter() - t0)
                row[f"{name}_ms"] = round(best * 1e3, 3)
            if "direct" in res:
                if not (res["fft"] == res["direct"]).all():
                    raise RuntimeError(f"full-vector C4 routes differ at L={L}")
                row["speedup"] = round(row["direct_ms"] / row["fft_ms"], 1)
            out[f"L{L}"] = row
            log(json.dumps({"shells_probe_progress": L, **row}))
            g.close()
    finally:
        ea.set_shell_route(ea.SHELLS_AUTO)
    return out


def exchange_probe(words: int = 64, iters: int = 2000) -> dict:
    """One-way latency of the slab path's exchange (64-bit {word, epoch}
    entries, agent-scope stores and polled loads) between two workgroups on
    one XCD and on two (libea_probe.so, ea_probe_exchange): `words` entries
    per message, one per lane as in the slab path, averaged over `iters`."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1411_5512_amd", "libea_probe.so"))
    lib.ea_probe_exchange.restype = ctypes.c_int
    lib.ea_probe_exchange.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_uint32)]
    out = {"words": words, "messages": iters}
    for partner in (8, 1):  # workgroups are dealt to the eight XCDs in turn
        us = ctypes.c_double(0.0)
        xcc = (ctypes.c_uint32 * 2)()
        rc = lib.ea_probe_exchange(partner, words, iters, ctypes.byref(us), xcc)
        if rc != 0:
            raise RuntimeError(f"ea_probe_exchange(partner={partner}) failed: {rc}")
        key = "same_xcd" if xcc[0] == xcc[1] else "other_xcd"
        out[f"one_way_us_{key}"] = round(us.value, 3)
        out[f"xcds_{key}"] = [int(xcc[0]), int(xcc[1])]
    return out


def bench_msc(ea, torch, job, burst: int):
    """The multispin-coded batch (asynchronous multispin coding, shared random
    words) on the paper's production configuration: the whole schedule once
    (sweeps, snapshots, measurements; wall clock), then a burst of sweeps
    timed with events on the batch's stream for the half-step launch."""
    warm = ea.Msc(job.L, job.n_samples, job.p, job.T, seed=job.seed, sample0=job.sample, shared=0)
    warm.sweep(64)  # loads the kernels; each handle captures its own graph on its first long run
    warm.close()
    g = ea.Msc(job.L, job.n_samples, job.p, job.T, seed=job.seed, sample0=job.sample, shared=0,
               n_slots=len(job.tw))
    g.sync()
    w0 = time.perf_counter()
    t_now, n_meas = 0, 0
    for t, slots, meas in job.events():
        g.sweep(t - t_now)
        t_now = t
        for k in slots:
            g.snapshot(k)
        if meas:
            g.measure()
            n_meas += 1
    g.sweep(job.n_sweeps - t_now)
    g.sync()
    run_s = time.perf_counter() - w0
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(g.stream)
    g.sweep(burst)
    b1.record(g.stream)
    torch.cuda.synchronize()
    half_us = b0.elapsed_time(b1) * 1e3 / (2 * burst)
    g.close()
    L, B = job.L, job.n_samples
    words = B // min(B, 32) * (L // 2) * L * L  # words per plane (P) times word sets
    alg_bytes = 48 * words  # per half-step: 2 replicas x (read 2 planes, write 1) + 6 coupling planes, 4 B each
    flips_half = L ** 3 * B  # both replicas, half the sites each
    gbs = alg_bytes / (half_us * 1e-6) / 1e9
    # the record holds the counters of the 64-sample batch at L = 128
    traffic, traffic_src = (measured_traffic(MSC_TRAFFIC_FILE, MSC_SOURCES) if (L, B) == (128, 64)
                            else (None, "no counter record for this batch"))
    return {
        "workload": f"multispin-coded batch: L={L}, {B} samples x 2 replicas sharing one random word per "
                    f"site and sweep, p={job.p}, T={job.T}, {job.n_sweeps} sweeps, {n_meas} measurements, "
                    f"tw={job.tw}; one launch per half-step",
        "ps_per_flip": round(run_s / job.flips * 1e12, 4),
        "ps_per_flip_sweeps": round(half_us * 1e-6 / flips_half * 1e12, 4),
        "half_step_avg_us": round(half_us, 3),
        "roofline": {"bound": "hbm", "kernel": "msc_half_step_kernel", "achieved": round(gbs, 1),
                     "peak": 8000.0, "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                     "alg_bytes_per_launch": alg_bytes, "traffic": traffic, "traffic_source": traffic_src,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_frac": (round(traffic / (half_us * 1e-6) / 1e9 / 8000.0, 4) if traffic else None)},
        "vs_paper_8ps": round(8.0 / (run_s / job.flips * 1e12), 1),
    }


def bench_crossover(ea, torch, jobs, sample_sweeps: int, burst: int):
    """The crossover runs (five L = 128 samples, one per p, 10^6 sweeps and 30
    measurements each) with their own schedules, grouped: one slab launch for
    all five between events (wall clock, measurements included).  Beside it a
    burst of grouped sweeps timed with events (the kernel alone) and, for
    context, the runs one after the other on a bounded sample of
    `sample_sweeps` sweeps."""
    flips = sum(j.flips for j in jobs)
    ea.run_group(jobs[:1])  # warm-up: kernels and the plain packing
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ea.run_group(jobs)
    torch.cuda.synchronize()
    grouped = time.perf_counter() - w0
    sims = [ea.Sim(j.L, j.p, j.T, seed=j.seed, sample=j.sample) for j in jobs]
    ea.sweep_group(sims, 64)
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(sims[0].stream)
    ea.sweep_group(sims, burst)
    b1.record(sims[0].stream)
    torch.cuda.synchronize()
    sweep_us = b0.elapsed_time(b1) * 1e3 / burst
    plan = sims[0].slab_plan
    for s_ in sims:
        s_.close()
    flips_sweep = sum(2 * j.L ** 3 for j in jobs)
    alu = ALG_OPS_PER_FLIP * flips_sweep / (sweep_us * 1e-6) / 1e12
    from paper_1411_5512_amd import workloads as wl
    small = wl.crossover_jobs(sample_sweeps)
    w0 = time.perf_counter()
    for j in small:
        ea.run_group([j])
    torch.cuda.synchronize()
    separate = time.perf_counter() - w0
    return {
        "workload": f"{len(jobs)} plain runs, L={jobs[0].L}, p in {[j.p for j in jobs]}, T={jobs[0].T}, "
                    f"{jobs[0].n_sweeps} sweeps, {len(jobs[0].meas_t)} measurements each",
        "ps_per_flip_grouped": round(grouped / flips * 1e12, 4),
        "wall_s_grouped": round(grouped, 3),
        "sweep_avg_us_grouped": round(sweep_us, 3),
        "ps_per_flip_sweeps_grouped": round(sweep_us * 1e-6 / flips_sweep * 1e12, 4),
        "alu_frac_grouped": round(alu / VALU_PEAK_TOPS, 5),
        "slab_plan_alone": {"slabs_per_replica": plan[0], "ghost_planes": plan[1]},
        "ps_per_flip_one_by_one": round(separate / sum(j.flips for j in small) * 1e12, 4),
        "one_by_one_sample": f"the same five runs one after the other, {sample_sweeps} sweeps each",
    }


SERVE_SIZES = (16, 24, 32, 48, 64, 96, 128)


def _serve(ea, stream, gap_s: float, budget: int, what: str):
    """Submit `stream` ((arrival in mean gaps, job) pairs) to a server at the
    given mean gap and wait for every job; progress lines on stderr."""
    srv = ea.Server(hbm_budget=budget, max_resident=512)
    srv.start()
    t0 = time.perf_counter()
    last = t0
    for i, (arrival, job) in enumerate(stream):
        delay = t0 + arrival * gap_s - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        srv.submit(job)
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            log(f"{what}: {i + 1}/{len(stream)} submitted, {srv.stats()['completed']} done, "
                f"{last - t0:.0f} s")
    while True:
        try:
            srv.drain(20.0)
            break
        except ea.EAError as e:
            if e.status != ea.abi.EA_ERR_BUSY or time.perf_counter() - t0 > 3600:
                raise
            log(f"{what}: {srv.stats()['completed']}/{len(stream)} done, {time.perf_counter() - t0:.0f} s")
    wall = time.perf_counter() - t0
    srv.stop()
    st = srv.stats()
    srv.close()
    return st, wall


def bench_serving(ea, torch, wl, n_jobs: int, load: float, sweep_hi: int, calib_jobs: int = 100):
    """Poisson stream of jobs (L uniform over {16,...,128}, p ~ U[0.1,0.5],
    T ~ U[0.5,1.2], sweeps log-uniform in [1e3, sweep_hi], log-spaced
    schedules) offered at `load` times the serving form's own capacity,
    measured first on a burst of `calib_jobs` jobs of the same distribution
    (another seed) submitted at once; continuous batching with admission by
    an HBM budget."""
    budget = 1 << 30
    calib = wl.serve_jobs(n_jobs=calib_jobs, gen_seed=6, sweep_range=(1_000, sweep_hi), sizes=SERVE_SIZES)
    st, wall = _serve(ea, [(0.0, j) for _, j in calib], 0.0, budget, "serving capacity burst")
    ps_capacity = wall / sum(j.flips for _, j in calib) * 1e12
    stream = wl.serve_jobs(n_jobs=n_jobs, sweep_range=(1_000, sweep_hi), sizes=SERVE_SIZES)
    total = sum(j.flips for _, j in stream)
    gap_s = total * ps_capacity * 1e-12 / len(stream) / load
    st, wall = _serve(ea, stream, gap_s, budget, f"serving at load {load}")
    full = n_jobs >= 2000 and sweep_hi >= 1_000_000
    return {
        "config5": full,
        "sample": ("the serving configuration as stated (2000 jobs, sweeps log-uniform in [1e3, 1e6])" if full else
                   f"a bounded sample of the serving configuration: {n_jobs} of its 2000 jobs, sweeps "
                   f"log-uniform in [1e3, {sweep_hi:.0e}] instead of [1e3, 1e6]"),
        "workload": f"{n_jobs} Poisson arrivals (mean gap {gap_s * 1e3:.2f} ms = load {load} of the capacity "
                    f"measured on a burst of {calib_jobs} jobs), L uniform in {{16,24,32,48,64,96,128}} "
                    f"(L > 64 as slab launches after each epoch's batched launch), p~U[0.1,0.5], T~U[0.5,1.2], "
                    f"sweeps log-uniform in [1e3,{sweep_hi:.0e}], 20 log-spaced measurements; HBM budget "
                    f"{budget >> 20} MiB",
        "p50_latency_s": round(st["p50_latency_s"], 4),
        "p99_latency_s": round(st["p99_latency_s"], 4),
        "mean_latency_s": round(st["mean_latency_s"], 4),
        "max_latency_s": round(st["max_latency_s"], 4),
        "ps_per_flip_busy": round(st["ps_per_flip"], 4),
        "ps_per_flip_wall": round(wall / total * 1e12, 4),
        "ps_per_flip_capacity_burst": round(ps_capacity, 4),
        "flips": total,
        "epochs": int(st["epochs"]),
        "small_jobs_on_slabs": int(st["streamed_small"]),
        "jobs_moved_to_slabs": int(st["moved"]),
        "hbm_peak_mib": round(st["hbm_peak"] / 2 ** 20, 1),
        "wall_s": round(wall, 3),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--jobs", type=int, default=256, help="jobs in the batched workload")
    ap.add_argument("--sweeps", type=int, default=100_000, help="sweeps per job")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--burst", type=int, default=2048, help="sweeps in the plain kernel-timing burst")
    ap.add_argument("--cpu-sweeps", type=int, default=60, help="oracle sweeps for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-agg-sweeps", type=int, default=20,
                    help="sweeps per process of the all-core oracle rate (0 = skip)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-shells", action="store_true", help="skip the full-vector C4 leg")
    ap.add_argument("--no-autotune", action="store_true", help="run every size with its default configuration")
    ap.add_argument("--serve-jobs", type=int, default=300, help="jobs in the serving leg (0 = skip)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="offered load of the serving leg")
    ap.add_argument("--serve-load2", type=float, default=0.5,
                    help="a second, lighter offered load reported beside it (0 = skip)")
    ap.add_argument("--serve-sweeps", type=int, default=10_000, help="upper end of the serving sweep range")
    ap.add_argument("--msc-sweeps", type=int, default=10_000,
                    help="sweeps of the multispin-coded batch (0 = skip that leg)")
    ap.add_argument("--msc-samples", type=int, default=64, help="samples of the multispin-coded batch")
    ap.add_argument("--msc-burst", type=int, default=1024, help="sweeps in its kernel-timing burst")
    ap.add_argument("--msc-only", action="store_true", help="run only the multispin-coded leg and print it")
    ap.add_argument("--crossover-only", action="store_true", help="run only the crossover leg and print it")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg(s) and print them (e.g. --serve-jobs 2000 --serve-sweeps "
                         "1000000 for the serving configuration as stated)")
    ap.add_argument("--plain-only", action="store_true", help="run only the mid-size plain leg and print it")
    ap.add_argument("--crossover-sweeps", type=int, default=1_000_000,
                    help="sweeps of each crossover run in the grouped-plain leg (0 = skip)")
    ap.add_argument("--crossover-sample-sweeps", type=int, default=10_000,
                    help="sweeps of the bounded one-after-the-other sample beside it")
    ap.add_argument("--alu-probe", action="store_true",
                    help="only measure the lane rate of v_mad_u64_u32, v_bitop3_b32 and whole Philox4x32-10 "
                         "blocks against the integer-ALU peak (the roofline's op count) and exit")
    ap.add_argument("--shells-probe", action="store_true",
                    help="only time the full-vector C4 shells (every displacement) by the FFT and the direct "
                         "route at L = 32, 64, 128, 256, check that they agree, and exit")
    ap.add_argument("--shells-probe-l", type=int, default=0, help="with --shells-probe: this L only")
    ap.add_argument("--shells-fft-only", action="store_true", help="with --shells-probe: the FFT route only")
    ap.add_argument("--xchg-probe", action="store_true",
                    help="only measure the one-way latency of the slab path's exchange between two workgroups "
                         "on one XCD and on two, and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (a known-size kernel "
                         "for calibrating hardware byte counters) and exit")
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

    if args.alu_probe:
        print(json.dumps({"alu_probe": alu_probe()}), flush=True)
        return

    if args.shells_probe:
        sizes = (args.shells_probe_l,) if args.shells_probe_l else (32, 64, 128, 256)
        print(json.dumps({"shells_probe": shells_probe(ea, sizes, direct_sizes=() if args.shells_fft_only
                                                       else sizes)}), flush=True)
        return

    if args.xchg_probe:
        print(json.dumps({"exchange_probe": {str(w): exchange_probe(w) for w in (64, 256)}}), flush=True)
        return

    if args.copy_probe_mib:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "read": n, "written": n}), flush=True)
        return

    if args.serve_only:
        res = {"serving": bench_serving(ea, torch, wl, args.serve_jobs, args.serve_load, args.serve_sweeps)}
        if args.serve_load2 > 0:
            res["serving_light"] = bench_serving(ea, torch, wl, args.serve_jobs, args.serve_load2,
                                                 args.serve_sweeps)
        print(json.dumps(res), flush=True)
        return
    if args.crossover_only:
        print(json.dumps({"crossover": bench_crossover(ea, torch, wl.crossover_jobs(args.crossover_sweeps),
                                                       args.crossover_sample_sweeps, args.burst)}), flush=True)
        return
    if args.plain_only:
        print(json.dumps({"plain": bench_plain(ea, torch, wl.mid_job(args.sweeps), args.plain_steps, args.burst)}),
              flush=True)
        return

    if args.msc_only:
        print(json.dumps({"msc": bench_msc(ea, torch, wl.msc_job(args.msc_sweeps, args.msc_samples),
                                           args.msc_burst)}), flush=True)
        return

    jobs = wl.batch_jobs(n_jobs=args.jobs, n_sweeps=args.sweeps)
    flips_per_step = sum(j.flips for j in jobs)
    Ls = sorted({j.L for j in jobs})
    tuned = {}
    if not args.no_autotune:
        for L in Ls:  # untimed: probes every candidate, keeps the bit-exact fastest
            tuned[L] = ea.tune(L)["chosen"]
            log(f"autotune L={L}: {tuned[L]}")
    batch = ea.Batch(jobs, autotune=not args.no_autotune)
    stream = batch.stream
    batch.capture()  # reset + full run as one hipGraph

    for i in range(args.warmup):
        batch.replay()
        log(f"warmup {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    run_ms = []
    w0 = time.perf_counter()
    for i in range(args.steps):
        ev0.record(stream)
        batch.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        run_ms.append(ev0.elapsed_time(ev1))
        log(f"step {i + 1}/{args.steps} done ({run_ms[-1]:.1f} ms for the graph: reset + batch launch)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = wall * 1e3 / args.steps
    ps_per_flip = ms_per_step * 1e-3 / flips_per_step * 1e12
    launch_s = sum(run_ms) / len(run_ms) * 1e-3
    achieved = ALG_OPS_PER_FLIP * flips_per_step / launch_s / 1e12

    # the results are on the device; read them back once, outside the timing,
    # and check the identity C(t_w, t_w) = 1 on every job
    for j, job in enumerate(jobs):
        for k, t in enumerate(job.meas_t):
            if t in job.tw:
                o = batch.result(j, k, c4=False)
                slot = job.tw.index(t)
                assert list(o.autocorr[:, slot]) == [job.L ** 3] * 2, (j, k)
    n_results = sum(len(j.meas_t) for j in jobs)

    traffic, traffic_src = measured_traffic()
    record, _ = measured_record()
    valu_issue = float(record["valu_issue"]) if record and "valu_issue" in record else None
    alg_bytes = algorithmic_bytes(jobs)
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
            "workload": f"batched form: {len(jobs)} samples x 2 replicas, L in {Ls}, p in {{0.5,0.3,0.2}}, "
                        f"T in {{0.6,0.8,1.0}}, seeds 0..{len(jobs) - 1}, {args.sweeps} sweeps each, "
                        f"20 log-spaced measurements + tw {{1e2,1e3,1e4}}, one persistent launch (graph: "
                        f"device-side regeneration of every job + the launch)",
            "form": "batched",
            "jobs": len(jobs),
            "sweeps": args.sweeps,
            "flips_per_step": flips_per_step,
            "measurements_per_step": n_results,
            "launch_config": {str(L): (f"{c['words_per_row']} words/row, {c['threads']} threads, "
                                       f"{c['select']} select") for L, c in tuned.items()} or "default",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "batch_kernel",
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s (32-bit lane-op slots)",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": traffic,
            "launch_ms": round(launch_s * 1e3, 3),
            "alg_ops_per_flip": ALG_OPS_PER_FLIP,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_source": traffic_src,
            "alg_bytes_per_launch": alg_bytes,
            "valu_issue_measured": valu_issue,  # SQ_INSTS_VALU over the device's issue slots (record)
            "hbm_frac": round(((traffic or alg_bytes) / launch_s / 1e9) / 8000.0, 5),
            "flips_per_launch": flips_per_step,
            "pricing": (f"{ALG_OPS_PER_FLIP:g} lane-op slots per flip (a quarter Philox4x32-10 block with its "
                        f"multiply-adds at the half rate --alu-probe measures, plus the compare) against "
                        f"{VALU_PEAK_TOPS:.2f} T slots/s; the earlier pricing, 11 ops per flip against a 16-lane "
                        f"39.32 T ops/s, gives {11 * flips_per_step / launch_s / 1e12 / 39.32:.3f} for the same "
                        f"launch"),
        },
    }
    batch.close()

    if args.serve_jobs:
        log("serving form ...")
        out["serving"] = bench_serving(ea, torch, wl, args.serve_jobs, args.serve_load, args.serve_sweeps)
        if args.serve_load2 > 0:
            log(f"serving form at load {args.serve_load2} ...")
            out["serving_light"] = bench_serving(ea, torch, wl, args.serve_jobs, args.serve_load2,
                                                 args.serve_sweeps)
    if args.msc_sweeps:
        log("multispin-coded batch ...")
        out["msc"] = bench_msc(ea, torch, wl.msc_job(args.msc_sweeps, args.msc_samples), args.msc_burst)
    if args.crossover_sweeps:
        log("crossover runs, grouped ...")
        out["crossover"] = bench_crossover(ea, torch, wl.crossover_jobs(args.crossover_sweeps),
                                           args.crossover_sample_sweeps, args.burst)
    if not args.no_plain:
        log("plain form ...")
        plain = bench_plain(ea, torch, wl.mid_job(args.sweeps), args.plain_steps, args.burst)
        out["plain"] = plain
        out["batched_speedup_vs_plain"] = round(plain["ps_per_flip"] / ps_per_flip, 2)
    if not args.no_shells:
        log("full-vector C4 shells ...")
        out["shells"] = {"workload": "ea_c4_shells over every displacement (3 (L/2)^2 + 1 shells) of one run "
                                     "after 20 sweeps, one synchronous call, best of 3",
                         "per_pass_roofline": "profiles/fft_shells_L256.md",
                         **shells_probe(ea, sizes=(128, 256), direct_sizes=(128,))}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        n_cpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(wl.mid_job(args.sweeps), args.cpu_sweeps, min(16, n_cpu),
                                           args.cpu_agg_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
