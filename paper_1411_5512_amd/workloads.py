"""Seeded synthetic workloads: run parameters and measurement schedules.

This module only describes *what* to run (lattice size, coupling probability,
temperature, seeds, sweep counts and the times at which to snapshot and
measure); it holds none of the simulation's arithmetic.  Tests, the benchmark
and the smoke check use it to hand identical inputs to the GPU library and to
the CPU oracle.

The paper's production runs are 128^3 samples with two replicas quenched to
T = 0.8 for 10^8 sweeps, across the spin-glass/ferromagnet crossover (Sec. IV).
The workloads below are scaled-down synthetic stand-ins of that shape; the
couplings and initial spins themselves are drawn inside the library and the
oracle from (seed, sample).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def log_schedule(n_sweeps: int, k: int) -> list[int]:
    """k log-spaced times in [1, n_sweeps]: round(10^(i log10(n) / (k-1))),
    de-duplicated and sorted."""
    if n_sweeps < 1 or k < 1:
        return []
    if k == 1:
        return [int(n_sweeps)]
    lg = math.log10(n_sweeps)
    ts = {int(math.floor(10 ** (i * lg / (k - 1)) + 0.5)) for i in range(k)}
    return sorted(t for t in ts if 1 <= t <= n_sweeps)


@dataclass
class Job:
    """One run: a coupling sample with two replicas and its schedule."""

    L: int
    p: float
    T: float
    seed: int
    sample: int = 0
    n_sweeps: int = 0
    meas_t: list = field(default_factory=list)   # sorted measurement times
    tw: list = field(default_factory=list)       # sorted snapshot (waiting) times
    n_samples: int = 1                           # samples run together (multispin batch)

    @property
    def flips(self) -> int:
        """Attempted single-spin updates of the whole run (both replicas, every sample)."""
        return 2 * self.L ** 3 * self.n_sweeps * self.n_samples

    def events(self):
        """Chronological (time, snapshot_slots, measure) events."""
        times = sorted(set(self.meas_t) | set(self.tw))
        for t in times:
            slots = [k for k, w in enumerate(self.tw) if w == t]
            yield t, slots, t in self.meas_t


def small_job() -> Job:
    """L = 16, p = 0.5, T = 0.8, 1000 sweeps, measure at 10, 100, 1000, t_w = 100."""
    return Job(16, 0.5, 0.8, seed=1, sample=0, n_sweeps=1000, meas_t=[10, 100, 1000], tw=[100])


def mid_job(n_sweeps: int = 100_000) -> Job:
    """L = 64, p = 0.5, T = 0.7, 10^5 sweeps, 20 log-spaced measurements,
    t_w in {10^2, 10^3, 10^4}."""
    tw = [t for t in (100, 1000, 10_000) if t <= n_sweeps]
    meas = sorted(set(log_schedule(n_sweeps, 20)) | set(tw))
    return Job(64, 0.5, 0.7, seed=1, sample=0, n_sweeps=n_sweeps, meas_t=meas, tw=tw)


def crossover_jobs(n_sweeps: int = 1_000_000) -> list[Job]:
    """L = 128 at p in {0.5, 0.3, 0.25, 0.2, 0.15}, T = 0.7, one seed (nested
    couplings across p), 30 log-spaced measurements."""
    meas = log_schedule(n_sweeps, 30)
    tw = [t for t in (100, 10_000) if t <= n_sweeps]
    return [Job(128, p, 0.7, seed=1, sample=0, n_sweeps=n_sweeps,
                meas_t=sorted(set(meas) | set(tw)), tw=tw)
            for p in (0.5, 0.3, 0.25, 0.2, 0.15)]


def msc_job(n_sweeps: int = 10_000, n_samples: int = 64) -> Job:
    """The paper's production batch (Sec. IV): L = 128, p = 0.5, T = 0.8, the
    samples of one multispin word set (64 by default) sharing the random words,
    20 log-spaced measurements and t_w in {10^2, 10^3}.  `sample` is the
    first sample; the batch has n_samples of them."""
    tw = [t for t in (100, 1000) if t <= n_sweeps]
    meas = sorted(set(log_schedule(n_sweeps, 20)) | set(tw))
    return Job(128, 0.5, 0.8, seed=1, sample=0, n_sweeps=n_sweeps, meas_t=meas, tw=tw, n_samples=n_samples)


def batch_jobs(n_jobs: int = 256, n_sweeps: int = 100_000, gen_seed: int = 4) -> list[Job]:
    """Many independent samples of uneven size: job j has seed j; L, p, T are
    drawn uniformly from {24, 32, 48, 64}, {0.5, 0.3, 0.2}, {0.6, 0.8, 1.0}."""
    rng = np.random.default_rng(gen_seed)
    Ls = rng.choice([24, 32, 48, 64], size=n_jobs)
    ps = rng.choice([0.5, 0.3, 0.2], size=n_jobs)
    Ts = rng.choice([0.6, 0.8, 1.0], size=n_jobs)
    tw = [t for t in (100, 1000, 10_000) if t <= n_sweeps]
    meas = sorted(set(log_schedule(n_sweeps, 20)) | set(tw))
    return [Job(int(Ls[j]), float(ps[j]), float(Ts[j]), seed=j, sample=0, n_sweeps=n_sweeps,
                meas_t=list(meas), tw=list(tw)) for j in range(n_jobs)]


def serve_jobs(n_jobs: int = 2000, gen_seed: int = 5, sweep_range=(1_000, 1_000_000),
               sizes=(16, 24, 32, 48, 64, 96, 128)) -> list[tuple[float, Job]]:
    """Poisson job stream: (arrival offset in units of the mean gap, job).
    L uniform over sizes, p ~ U[0.1, 0.5], T ~ U[0.5, 1.2], sweeps
    log-uniform in sweep_range, 20 log-spaced measurements per job."""
    rng = np.random.default_rng(gen_seed)
    gaps = rng.exponential(1.0, size=n_jobs)
    arrivals = np.cumsum(gaps)
    out = []
    lo, hi = math.log(sweep_range[0]), math.log(sweep_range[1])
    for j in range(n_jobs):
        L = int(rng.choice(sizes))
        p = float(rng.uniform(0.1, 0.5))
        T = float(rng.uniform(0.5, 1.2))
        n = int(round(math.exp(rng.uniform(lo, hi))))
        meas = log_schedule(n, 20)
        tw = [t for t in (100, 1000) if t <= n]
        out.append((float(arrivals[j]), Job(L, p, T, seed=100_000 + j, sample=0, n_sweeps=n,
                                            meas_t=sorted(set(meas) | set(tw)), tw=tw)))
    return out
