"""MI355X (gfx950) checkerboard Metropolis ageing simulations of the 3D +-J
Edwards-Anderson model (Manssen & Hartmann, arXiv:1411.5512).

Python face of the C ABI in ``include/ea.h``: :class:`Sim` wraps one run (a
coupling sample with two replicas).  PyTorch, when importable with a GPU,
supplies the stream the library enqueues on and the device buffer it carves
its arrays from; all simulation work runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import abi
from .abi import EAError

__all__ = ["Sim", "Batch", "Server", "EAError", "thresholds", "footprint", "version", "tune", "sweep_group", "run_group", "Msc",
           "set_debug", "get_debug", "DEBUG_REVERSE", "DEBUG_ROTATE", "DEBUG_POISON",
           "set_shell_route", "get_shell_route", "SHELLS_AUTO", "SHELLS_DIRECT", "SHELLS_FFT"]


def version() -> str:
    return abi.lib().ea_version().decode()


def thresholds(T: float) -> np.ndarray:
    out = np.zeros(3, dtype=np.uint32)
    abi.check(abi.lib().ea_thresholds(float(T), abi.ptr(out, ctypes.c_uint32)))
    return out


DEBUG_REVERSE, DEBUG_ROTATE, DEBUG_POISON = 1, 2, 4


def set_debug(flags: int = 0, seed: int = 0) -> None:
    """Race and order debug mode (ea_set_debug): reversed and/or rotated
    workgroup order, LDS poisoned before the persistent kernels load; 0 = off.
    Applies to launches made after the call."""
    abi.check(abi.lib().ea_set_debug(int(flags), int(seed) & 0xFFFFFFFF))


def get_debug() -> tuple:
    f, s = ctypes.c_uint32(0), ctypes.c_uint32(0)
    abi.check(abi.lib().ea_get_debug(ctypes.byref(f), ctypes.byref(s)))
    return int(f.value), int(s.value)


SHELLS_AUTO, SHELLS_DIRECT, SHELLS_FFT = 0, 1, 2


def set_shell_route(route: int = SHELLS_AUTO) -> None:
    """Route of the full-vector C4 shells (ea_set_shell_route): automatic
    (FFT for L = 2^k or 3 2^k >= 64), direct bit counting, or FFT wherever
    L = 2^k or 3 2^k.  Both give identical results."""
    abi.check(abi.lib().ea_set_shell_route(int(route)))


def get_shell_route() -> int:
    r = ctypes.c_int32(0)
    abi.check(abi.lib().ea_get_shell_route(ctypes.byref(r)))
    return int(r.value)


def footprint(L: int, n_tw: int = 0, words_per_row: int = 0) -> int:
    """Device bytes of a plain run (words_per_row = 0: the library's packing)."""
    out = ctypes.c_size_t(0)
    if words_per_row == 0:
        abi.check(abi.lib().ea_footprint(int(L), int(n_tw), ctypes.byref(out)))
    else:
        cfg = abi.Config()
        cfg.L, cfg.n_tw_slots, cfg.words_per_row = int(L), int(n_tw), int(words_per_row)
        abi.check(abi.lib().ea_footprint_ex(ctypes.byref(cfg), ctypes.byref(out)))
    return int(out.value)


def tune(L: int, force: bool = False) -> dict:
    """Autotune the batched kernel for lattice size L (see ea_tune)."""
    chosen = abi.TuneChoice()
    tried = (abi.TuneChoice * 64)()
    n = ctypes.c_int32(0)
    abi.check(abi.lib().ea_tune(int(L), int(force), ctypes.byref(chosen), tried, 64, ctypes.byref(n)))

    def d(c):
        return {"words_per_row": c.words_per_row, "threads": c.threads,
                "select": "lds" if c.select == 0 else "reg", "ms": c.ms, "parity_ok": bool(c.parity_ok)}
    return {"chosen": d(chosen), "tried": [d(tried[i]) for i in range(n.value)]}


def tune_plain(L: int, force: bool = False) -> dict:
    """Autotune the plain form's bit packing for side L (see ea_tune_plain)."""
    rw = ctypes.c_int32(0)
    tried = (abi.TuneChoice * 64)()
    n = ctypes.c_int32(0)
    abi.check(abi.lib().ea_tune_plain(int(L), int(force), ctypes.byref(rw), tried, 64, ctypes.byref(n)))
    return {"words_per_row": rw.value,
            "tried": [{"words_per_row": tried[i].words_per_row, "threads": tried[i].threads, "ms": tried[i].ms,
                       "parity_ok": bool(tried[i].parity_ok)} for i in range(n.value)]}


def _torch_stream_and_buffer(nbytes: int, use_torch: bool):
    if not use_torch:
        return None, None
    try:
        import torch
    except ImportError:
        return None, None
    if not torch.cuda.is_available():
        return None, None
    # a stream of its own (default priority): graphs cannot be captured on the
    # legacy default stream, and timing events must sit on the run's stream
    stream = torch.cuda.Stream()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.current_stream().synchronize()
    return stream, buf


class Obs:
    """Integer observables of one measurement (see ``ea_obs`` in ea.h)."""

    __slots__ = ("t", "unsat", "mag", "overlap", "tw", "autocorr", "c4")

    def __init__(self, t, unsat, mag, overlap, tw, autocorr, c4):
        self.t, self.unsat, self.mag, self.overlap = t, unsat, mag, overlap
        self.tw, self.autocorr, self.c4 = tw, autocorr, c4

    def energy_per_spin(self, N: int) -> np.ndarray:
        return (2 * self.unsat - 3 * N) / N


class Sim:
    """One run: L^3 lattice, couplings with P(J=-1) = p, two replicas at T."""

    def __init__(self, L: int, p: float, T: float, seed: int, sample: int = 0,
                 n_slots: int = 0, use_torch: bool = True, words_per_row: int = 0):
        self.L, self.p, self.T = int(L), float(p), float(T)
        self.seed, self.sample, self.n_slots = int(seed), int(sample), int(n_slots)
        self.N = self.L ** 3
        self._h = None
        cfg = abi.Config()
        cfg.L, cfg.p, cfg.T = self.L, self.p, self.T
        cfg.seed, cfg.sample, cfg.n_tw_slots = self.seed, self.sample, self.n_slots
        cfg.words_per_row = int(words_per_row)
        need = ctypes.c_size_t(0)
        if abi.lib().ea_footprint_ex(ctypes.byref(cfg), ctypes.byref(need)) != 0:
            need = ctypes.c_size_t(0)  # invalid arguments: ea_create_ex reports them
        need = need.value
        self._stream, self._buf = _torch_stream_and_buffer(need, use_torch and need > 0)
        if self._stream is not None:
            cfg.stream = ctypes.c_void_p(self._stream.cuda_stream)
            base = self._buf.data_ptr()
            aligned = (base + 255) & ~255
            cfg.dev_buf = ctypes.c_void_p(aligned)
            cfg.dev_buf_bytes = need
        h = ctypes.c_void_p()
        abi.check(abi.lib().ea_create_ex(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    @property
    def words_per_row(self) -> int:
        rw = ctypes.c_int32(0)
        abi.check(abi.lib().ea_words_per_row(self._h, ctypes.byref(rw)))
        return rw.value

    def set_slab_plan(self, slabs: int = 0, ghost: int = 0):
        """Slab path of ea_sweep (see ea_set_slab_plan): slabs 0 = the
        library's choice, -1 = one launch per half-step, else that many
        z-slabs per replica with `ghost` ghost planes (0 = library's choice)."""
        abi.check(abi.lib().ea_set_slab_plan(self._h, int(slabs), int(ghost)))

    @property
    def slab_plan(self) -> tuple:
        """(slabs per replica, ghost planes) ea_sweep uses; (-1, 0) when off."""
        k, g = ctypes.c_int32(0), ctypes.c_int32(0)
        abi.check(abi.lib().ea_get_slab_plan(self._h, ctypes.byref(k), ctypes.byref(g)))
        return k.value, g.value

    # -- lifetime -------------------------------------------------------
    def close(self):
        if self._h is not None and self._h.value:
            abi.lib().ea_destroy(self._h)
        self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- dynamics -------------------------------------------------------
    @property
    def stream(self):
        return self._stream

    @property
    def time(self) -> int:
        t = ctypes.c_uint64(0)
        abi.check(abi.lib().ea_time(self._h, ctypes.byref(t)))
        return int(t.value)

    def set_time(self, t: int):
        abi.check(abi.lib().ea_set_time(self._h, int(t)))

    def reset(self, seed: int, sample: int = 0):
        """Restart in place for another sample (no allocation)."""
        abi.check(abi.lib().ea_reset(self._h, int(seed), int(sample)))
        self.seed, self.sample = int(seed), int(sample)

    def sweep(self, n: int = 1):
        abi.check(abi.lib().ea_sweep(self._h, int(n)))

    def snapshot(self, slot: int):
        abi.check(abi.lib().ea_snapshot(self._h, int(slot)))

    def sync(self):
        abi.check(abi.lib().ea_sync(self._h))

    def measure(self, c4: bool = True, autocorr: bool = True) -> Obs:
        o = abi.Obs()
        tw = np.zeros(max(self.n_slots, 1), dtype=np.uint64)
        ac = np.zeros((2, max(self.n_slots, 1)), dtype=np.int64)
        c4a = np.zeros((3, self.L // 2 + 1), dtype=np.int64)
        if autocorr and self.n_slots > 0:
            o.n_tw = self.n_slots
            o.tw = abi.ptr(tw, ctypes.c_uint64)
            o.autocorr = abi.ptr(ac, ctypes.c_int64)
        if c4:
            o.rmax = self.L // 2
            o.c4 = abi.ptr(c4a, ctypes.c_int64)
        abi.check(abi.lib().ea_measure(self._h, ctypes.byref(o)))
        ns = self.n_slots
        return Obs(int(o.t), np.array(o.unsat[:], dtype=np.int64), np.array(o.mag[:], dtype=np.int64),
                   int(o.overlap), tw[:ns].copy(), ac[:, :ns].copy(), c4a if c4 else None)

    def c4_shells(self, n_shells: int | None = None) -> np.ndarray:
        """Full-vector C4 sums by minimum-image squared distance (see
        ea_c4_shells); n_shells defaults to (L/2)^2 + 1 (|r| <= L/2)."""
        n = (self.L // 2) ** 2 + 1 if n_shells is None else int(n_shells)
        out = np.zeros(n, dtype=np.int64)
        abi.check(abi.lib().ea_c4_shells(self._h, n, abi.ptr(out, ctypes.c_int64)))
        return out

    # -- state ------------------------------------------------------------
    def spins(self, r: int) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.int8)
        abi.check(abi.lib().ea_get_spins(self._h, int(r), abi.ptr(out, ctypes.c_int8)))
        return out

    def set_spins(self, r: int, S):
        S = np.ascontiguousarray(S, dtype=np.int8)
        if S.size != self.N:
            raise ValueError("wrong spin count")
        abi.check(abi.lib().ea_set_spins(self._h, int(r), abi.ptr(S, ctypes.c_int8)))

    def bonds(self) -> np.ndarray:
        out = np.zeros(3 * self.N, dtype=np.int8)
        abi.check(abi.lib().ea_get_bonds(self._h, abi.ptr(out, ctypes.c_int8)))
        return out

    def set_bonds(self, J):
        J = np.ascontiguousarray(J, dtype=np.int8)
        if J.size != 3 * self.N:
            raise ValueError("wrong coupling count")
        abi.check(abi.lib().ea_set_bonds(self._h, abi.ptr(J, ctypes.c_int8)))


def sweep_group(sims, n: int = 1):
    """Advance several runs of one L and packing by n sweeps each in shared
    launches (see ea_sweep_group); same spins as separate Sim.sweep calls."""
    sims = list(sims)
    arr = (ctypes.c_void_p * max(len(sims), 1))(*[s._h.value if s._h is not None else None for s in sims])
    abi.check(abi.lib().ea_sweep_group(arr, len(sims), int(n)))


class Msc:
    """Multispin-coded batch (asynchronous multispin coding, Sec. III): the
    samples sample0 .. sample0 + n_samples - 1 of one L, p, T share one word per
    site and one random word per site and sweep (see ea_msc_* in ea.h)."""

    def __init__(self, L: int, n_samples: int, p: float, T: float, seed: int, sample0: int = 0,
                 shared: int = 0, n_slots: int = 0, use_torch: bool = True):
        self.L, self.n_samples, self.p, self.T = int(L), int(n_samples), float(p), float(T)
        self.seed, self.sample0, self.shared, self.n_slots = int(seed), int(sample0), int(shared), int(n_slots)
        self.N = self.L ** 3
        self._h = None
        cfg = abi.MscConfig()
        cfg.L, cfg.n_samples, cfg.p, cfg.T = self.L, self.n_samples, self.p, self.T
        cfg.seed, cfg.sample0, cfg.shared, cfg.n_tw_slots = self.seed, self.sample0, self.shared, self.n_slots
        need = ctypes.c_size_t(0)
        if abi.lib().ea_msc_footprint(ctypes.byref(cfg), ctypes.byref(need)) != 0:
            need = ctypes.c_size_t(0)  # invalid arguments: ea_msc_create reports them
        need = need.value
        self._stream, self._buf = _torch_stream_and_buffer(need, use_torch and need > 0)
        if self._stream is not None:
            cfg.stream = ctypes.c_void_p(self._stream.cuda_stream)
            cfg.dev_buf = ctypes.c_void_p((self._buf.data_ptr() + 255) & ~255)
            cfg.dev_buf_bytes = need
        h = ctypes.c_void_p()
        abi.check(abi.lib().ea_msc_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def footprint(L: int, n_samples: int, n_slots: int = 0) -> int:
        cfg = abi.MscConfig()
        cfg.L, cfg.n_samples, cfg.n_tw_slots = int(L), int(n_samples), int(n_slots)
        out = ctypes.c_size_t(0)
        abi.check(abi.lib().ea_msc_footprint(ctypes.byref(cfg), ctypes.byref(out)))
        return int(out.value)

    def close(self):
        if self._h is not None and self._h.value:
            abi.lib().ea_msc_destroy(self._h)
        self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return self._stream

    @property
    def time(self) -> int:
        t = ctypes.c_uint64(0)
        abi.check(abi.lib().ea_msc_time(self._h, ctypes.byref(t)))
        return int(t.value)

    def set_time(self, t: int):
        abi.check(abi.lib().ea_msc_set_time(self._h, int(t)))

    def sweep(self, n: int = 1):
        abi.check(abi.lib().ea_msc_sweep(self._h, int(n)))

    def snapshot(self, slot: int):
        abi.check(abi.lib().ea_msc_snapshot(self._h, int(slot)))

    def sync(self):
        abi.check(abi.lib().ea_msc_sync(self._h))

    def measure(self, c4: bool = True, autocorr: bool = True) -> list:
        B = self.n_samples
        objs = (abi.Obs * B)()
        bufs = [_obs_buffers(self.L, self.n_slots if autocorr else 0, c4, objs[b]) for b in range(B)]
        abi.check(abi.lib().ea_msc_measure(self._h, objs))
        ns = self.n_slots if autocorr else 0
        return [Obs(int(objs[b].t), np.array(objs[b].unsat[:], dtype=np.int64),
                    np.array(objs[b].mag[:], dtype=np.int64), int(objs[b].overlap),
                    bufs[b][0][:ns].copy(), bufs[b][1][:, :ns].copy(), bufs[b][2] if c4 else None)
                for b in range(B)]

    def c4_shells(self, sample: int, n_shells: int | None = None) -> np.ndarray:
        """Full-vector C4 sums by minimum-image squared distance of one
        sample (see ea_msc_c4_shells); n_shells defaults to (L/2)^2 + 1."""
        n = (self.L // 2) ** 2 + 1 if n_shells is None else int(n_shells)
        out = np.zeros(n, dtype=np.int64)
        abi.check(abi.lib().ea_msc_c4_shells(self._h, int(sample), n, abi.ptr(out, ctypes.c_int64)))
        return out

    def spins(self, b: int, r: int) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.int8)
        abi.check(abi.lib().ea_msc_get_spins(self._h, int(b), int(r), abi.ptr(out, ctypes.c_int8)))
        return out

    def set_spins(self, b: int, r: int, S):
        S = np.ascontiguousarray(S, dtype=np.int8)
        if S.size != self.N:
            raise ValueError(f"{S.size} spins given, {self.N} needed")
        abi.check(abi.lib().ea_msc_set_spins(self._h, int(b), int(r), abi.ptr(S, ctypes.c_int8)))

    def bonds(self, b: int) -> np.ndarray:
        out = np.zeros(3 * self.N, dtype=np.int8)
        abi.check(abi.lib().ea_msc_get_bonds(self._h, int(b), abi.ptr(out, ctypes.c_int8)))
        return out


def run_group(jobs, words_per_row: int = 0, use_torch: bool = True):
    """Run several plain jobs of one L together (see ea_sweep_group): every
    run follows its own schedule of snapshots and measurements, and between
    events all runs advance in shared launches.  `jobs` are workloads.Job-like
    (L, p, T, seed, sample, n_sweeps, meas_t, tw, events()).  Returns, per job,
    the list of Obs at its measurement times.  Same results as running each
    job alone."""
    jobs = list(jobs)
    if not jobs:
        return []
    sims = [Sim(j.L, j.p, j.T, seed=j.seed, sample=j.sample, n_slots=len(j.tw), use_torch=use_torch,
                words_per_row=words_per_row) for j in jobs]
    events = {}
    for i, j in enumerate(jobs):
        for te, slots, meas in j.events():
            events.setdefault(int(te), []).append((i, slots, meas))
        events.setdefault(int(j.n_sweeps), [])
    out = [[] for _ in jobs]
    t = 0
    for te in sorted(events):
        # the runs still going at te advance together
        live = [s for s, j in zip(sims, jobs) if j.n_sweeps >= te]
        if te > t:
            sweep_group(live, te - t)
            t = te
        for i, slots, meas in events[te]:
            for k in slots:
                sims[i].snapshot(k)
            if meas:
                out[i].append(sims[i].measure())
    for s in sims:
        s.sync()
        s.close()
    return out


def _job_struct(job, keep):
    """Fill an ea_job from a workloads.Job-like object; `keep` holds the
    schedule arrays alive for the duration of the call."""
    j = abi.Job()
    j.L, j.p, j.T = int(job.L), float(job.p), float(job.T)
    j.seed, j.sample, j.n_sweeps = int(job.seed), int(job.sample), int(job.n_sweeps)
    meas = np.ascontiguousarray(job.meas_t, dtype=np.uint64)
    tw = np.ascontiguousarray(job.tw, dtype=np.uint64)
    keep += [meas, tw]
    j.meas_t = abi.ptr(meas, ctypes.c_uint64) if meas.size else None
    j.n_meas = int(meas.size)
    j.tw = abi.ptr(tw, ctypes.c_uint64) if tw.size else None
    j.n_tw = int(tw.size)
    return j


def _obs_buffers(L, n_tw, c4, o):
    tw = np.zeros(max(n_tw, 1), dtype=np.uint64)
    ac = np.zeros((2, max(n_tw, 1)), dtype=np.int64)
    c4a = np.zeros((3, L // 2 + 1), dtype=np.int64)
    if n_tw:
        o.n_tw = n_tw
        o.tw = abi.ptr(tw, ctypes.c_uint64)
        o.autocorr = abi.ptr(ac, ctypes.c_int64)
    if c4:
        o.rmax = L // 2
        o.c4 = abi.ptr(c4a, ctypes.c_int64)
    return tw, ac, c4a


def _obs_from(o, n_tw, tw, ac, c4a, c4):
    return Obs(int(o.t), np.array(o.unsat[:], dtype=np.int64), np.array(o.mag[:], dtype=np.int64),
               int(o.overlap), tw[:n_tw].copy(), ac[:, :n_tw].copy(), c4a if c4 else None)


class Batch:
    """Many independent runs (L <= 64) in one persistent launch per span."""

    SPLIT_AUTO, SPLIT_NEVER, SPLIT_ALWAYS = 0, 1, 2

    def __init__(self, jobs, use_torch: bool = True, autotune: bool = False, split: int = 0):
        self.jobs = list(jobs)
        keep = []
        arr = (abi.Job * len(self.jobs))(*[_job_struct(j, keep) for j in self.jobs])
        opts = abi.BatchOpts()
        opts.autotune = 1 if autotune else 0
        opts.split = int(split)
        self._stream = None
        if use_torch:
            try:
                import torch
                if torch.cuda.is_available():
                    self._stream = torch.cuda.Stream()
                    opts.stream = ctypes.c_void_p(self._stream.cuda_stream)
            except ImportError:
                pass
        h = ctypes.c_void_p()
        abi.check(abi.lib().ea_batch_create(arr, len(self.jobs), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    def parts(self, j: int) -> int:
        """Workgroups per replica of job j: 1, or 2 if its replicas were split."""
        n = ctypes.c_int32(0)
        abi.check(abi.lib().ea_batch_parts(self._h, int(j), ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            abi.lib().ea_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return self._stream

    def reset(self):
        abi.check(abi.lib().ea_batch_reset(self._h))

    def run(self, t_stop: int | None = None):
        """Advance every job to min(t_stop, its n_sweeps) (default: the end)."""
        if t_stop is None:
            t_stop = max(j.n_sweeps for j in self.jobs)
        abi.check(abi.lib().ea_batch_run(self._h, int(t_stop)))

    def capture(self):
        """Capture reset + full run as a hipGraph (see replay)."""
        abi.check(abi.lib().ea_batch_capture(self._h))

    def replay(self):
        """Reset every job and run it to the end by replaying the graph."""
        abi.check(abi.lib().ea_batch_replay(self._h))

    def time(self, job: int) -> int:
        t = ctypes.c_uint64(0)
        abi.check(abi.lib().ea_batch_time(self._h, int(job), ctypes.byref(t)))
        return int(t.value)

    def result(self, job: int, k: int, c4: bool = True) -> Obs:
        J = self.jobs[job]
        o = abi.Obs()
        bufs = _obs_buffers(J.L, len(J.tw), c4, o)
        abi.check(abi.lib().ea_batch_result(self._h, int(job), int(k), ctypes.byref(o)))
        return _obs_from(o, len(J.tw), *bufs, c4)

    def c4_shells(self, job: int, k: int, n_shells: int | None = None) -> np.ndarray:
        """Full-vector C4 sums by minimum-image squared distance of job
        `job` at its measurement k (see ea_batch_c4_shells)."""
        L = self.jobs[job].L if 0 <= job < len(self.jobs) else 8  # a bad index: the library reports it
        n = (L // 2) ** 2 + 1 if n_shells is None else int(n_shells)
        out = np.zeros(n, dtype=np.int64)
        abi.check(abi.lib().ea_batch_c4_shells(self._h, int(job), int(k), n, abi.ptr(out, ctypes.c_int64)))
        return out

    def spins(self, job: int, r: int) -> np.ndarray:
        out = np.zeros(self.jobs[job].L ** 3, dtype=np.int8)
        abi.check(abi.lib().ea_batch_get_spins(self._h, int(job), int(r), abi.ptr(out, ctypes.c_int8)))
        return out


JOB_PENDING, JOB_RUNNING, JOB_DONE = 0, 1, 2


class Server:
    """Continuous batching of a job stream (see ea_server_* in ea.h)."""

    def __init__(self, hbm_budget: int, max_resident: int = 512, max_pending: int = 100000,
                 epoch_site_sweeps: int = 0, use_torch: bool = True):
        opts = abi.ServerOpts()
        opts.hbm_budget = int(hbm_budget)
        opts.max_resident = int(max_resident)
        opts.max_pending = int(max_pending)
        opts.epoch_site_sweeps = int(epoch_site_sweeps)
        self._stream = None
        if use_torch:
            try:
                import torch
                if torch.cuda.is_available():
                    self._stream = torch.cuda.Stream()
                    opts.stream = ctypes.c_void_p(self._stream.cuda_stream)
            except ImportError:
                pass
        h = ctypes.c_void_p()
        abi.check(abi.lib().ea_server_create(ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.jobs = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            abi.lib().ea_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return self._stream

    @staticmethod
    def footprint(job) -> int:
        keep = []
        j = _job_struct(job, keep)
        out = ctypes.c_size_t(0)
        abi.check(abi.lib().ea_server_footprint(ctypes.byref(j), ctypes.byref(out)))
        return int(out.value)

    def submit(self, job) -> int:
        keep = []
        j = _job_struct(job, keep)
        jid = ctypes.c_uint64(0)
        abi.check(abi.lib().ea_server_submit(self._h, ctypes.byref(j), ctypes.byref(jid)))
        self.jobs[int(jid.value)] = job
        return int(jid.value)

    def step(self) -> bool:
        p = ctypes.c_int32(0)
        abi.check(abi.lib().ea_server_step(self._h, ctypes.byref(p)))
        return bool(p.value)

    def start(self):
        abi.check(abi.lib().ea_server_start(self._h))

    def stop(self):
        abi.check(abi.lib().ea_server_stop(self._h))

    def drain(self, timeout_s: float = 600.0):
        abi.check(abi.lib().ea_server_drain(self._h, float(timeout_s)))

    def poll(self, jid: int) -> int:
        st = ctypes.c_int32(0)
        abi.check(abi.lib().ea_server_poll(self._h, int(jid), ctypes.byref(st)))
        return int(st.value)

    def result(self, jid: int, k: int, c4: bool = True) -> Obs:
        J = self.jobs[jid]
        o = abi.Obs()
        bufs = _obs_buffers(J.L, len(J.tw), c4, o)
        abi.check(abi.lib().ea_server_result(self._h, int(jid), int(k), ctypes.byref(o)))
        return _obs_from(o, len(J.tw), *bufs, c4)

    def latency(self, jid: int) -> float:
        v = ctypes.c_double(0)
        abi.check(abi.lib().ea_server_latency(self._h, int(jid), ctypes.byref(v)))
        return float(v.value)

    def release(self, jid: int):
        abi.check(abi.lib().ea_server_release(self._h, int(jid)))
        self.jobs.pop(jid, None)

    def stats(self) -> dict:
        r = abi.ServerReport()
        abi.check(abi.lib().ea_server_stats(self._h, ctypes.byref(r)))
        return {name: getattr(r, name) for name, _ in abi.ServerReport._fields_}
