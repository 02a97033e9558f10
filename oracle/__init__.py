"""Plain CPU oracle for the checkerboard Metropolis ageing simulation.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg load this; the product library never does.  The arithmetic
lives in ``ea_oracle.c`` (plain C, int8 spins, one site at a time); this module
only builds it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ea_oracle.c")
LIB = os.path.join(HERE, "libea_oracle.so")

TAG_METRO, TAG_BOND, TAG_INIT, TAG_SHARED = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no SIMD intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Obs(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_uint64),
        ("unsat", ctypes.c_int64 * 2),
        ("mag", ctypes.c_int64 * 2),
        ("overlap", ctypes.c_int64),
        ("autocorr", ctypes.POINTER(ctypes.c_int64)),
        ("c4", ctypes.POINTER(ctypes.c_int64)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i8p = ctypes.POINTER(ctypes.c_int8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.eao_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.eao_philox4x32_10.restype = None
        L.eao_site_word.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        L.eao_site_word.restype = ctypes.c_uint32
        L.eao_thresholds.argtypes = [ctypes.c_double, u32p]
        L.eao_thresholds.restype = None
        L.eao_colour.argtypes = [ctypes.c_int, ctypes.c_int64]
        L.eao_colour.restype = ctypes.c_int
        L.eao_half_index.argtypes = [ctypes.c_int, ctypes.c_int64]
        L.eao_half_index.restype = ctypes.c_int64
        L.eao_energy.argtypes = [ctypes.c_int, i8p, i8p]
        L.eao_energy.restype = ctypes.c_int64
        L.eao_delta_e.argtypes = [ctypes.c_int, i8p, i8p, ctypes.c_int64]
        L.eao_delta_e.restype = ctypes.c_int
        L.eao_create.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
        L.eao_create.restype = ctypes.c_void_p
        L.eao_destroy.argtypes = [ctypes.c_void_p]
        L.eao_destroy.restype = None
        L.eao_L.argtypes = [ctypes.c_void_p]
        L.eao_L.restype = ctypes.c_int
        L.eao_time.argtypes = [ctypes.c_void_p]
        L.eao_time.restype = ctypes.c_uint64
        L.eao_set_time.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.eao_set_time.restype = None
        L.eao_share_noise.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.eao_share_noise.restype = None
        L.eao_sweep.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.eao_sweep.restype = None
        L.eao_half_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.eao_half_step.restype = None
        L.eao_half_step_order.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p]
        L.eao_half_step_order.restype = None
        L.eao_snapshot.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.eao_snapshot.restype = ctypes.c_int
        L.eao_snapshot_time.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.eao_snapshot_time.restype = ctypes.c_uint64
        L.eao_measure.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Obs)]
        L.eao_c4_shells.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p]
        L.eao_c4_shells.restype = None
        L.eao_measure.restype = None
        for name in ("eao_get_spins", "eao_set_spins"):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int, i8p]
            getattr(L, name).restype = None
        for name in ("eao_get_bonds", "eao_set_bonds"):
            getattr(L, name).argtypes = [ctypes.c_void_p, i8p]
            getattr(L, name).restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().eao_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return out


def site_word(seed, sample, tag, aux, colour, replica, h) -> int:
    return int(lib().eao_site_word(seed, sample, tag, aux, colour, replica, h))


def thresholds(T: float) -> np.ndarray:
    out = np.zeros(3, dtype=np.uint32)
    lib().eao_thresholds(float(T), _ptr(out, ctypes.c_uint32))
    return out


def colour(L: int, s: int) -> int:
    return int(lib().eao_colour(L, s))


def half_index(L: int, s: int) -> int:
    return int(lib().eao_half_index(L, s))


def energy(L: int, S: np.ndarray, J: np.ndarray) -> int:
    S = np.ascontiguousarray(S, dtype=np.int8)
    J = np.ascontiguousarray(J, dtype=np.int8)
    return int(lib().eao_energy(L, _ptr(S, ctypes.c_int8), _ptr(J, ctypes.c_int8)))


def delta_e(L: int, S: np.ndarray, J: np.ndarray, s: int) -> int:
    S = np.ascontiguousarray(S, dtype=np.int8)
    J = np.ascontiguousarray(J, dtype=np.int8)
    return int(lib().eao_delta_e(L, _ptr(S, ctypes.c_int8), _ptr(J, ctypes.c_int8), s))


class Obs:
    """Integer observables of one measurement (see ea_oracle.h)."""

    def __init__(self, t, unsat, mag, overlap, autocorr, c4):
        self.t = t
        self.unsat = unsat          # (2,)
        self.mag = mag              # (2,)
        self.overlap = overlap
        self.autocorr = autocorr    # (2, n_slots)
        self.c4 = c4                # (3, L/2+1)

    def as_tuple(self):
        return (self.t, tuple(self.unsat), tuple(self.mag), self.overlap,
                tuple(map(tuple, self.autocorr)), tuple(map(tuple, self.c4)))


def shared_batch(L, p, T, seed, sample0, n_samples, shared_id, n_slots=0):
    """The samples sample0 .. sample0 + n_samples - 1 that one multispin word
    holds (Sec. III): separate runs whose Metropolis words all come from the
    shared stream shared_id."""
    sims = [Sim(L, p, T, seed, sample0 + b, n_slots) for b in range(n_samples)]
    for s in sims:
        s.share_noise(shared_id)
    return sims


class Sim:
    """One disorder sample with two replicas, run by the oracle."""

    def __init__(self, L, p, T, seed, sample=0, n_slots=0):
        self.L, self.p, self.T = int(L), float(p), float(T)
        self.seed, self.sample, self.n_slots = int(seed), int(sample), int(n_slots)
        self.N = self.L ** 3
        self.shared = None
        h = lib().eao_create(self.L, self.p, self.T, self.seed, self.sample, self.n_slots)
        if not h:
            raise ValueError(f"oracle rejected L={L} p={p} T={T} n_slots={n_slots}")
        self._h = h

    def close(self):
        if self._h:
            lib().eao_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self) -> int:
        return int(lib().eao_time(self._h))

    def set_time(self, t: int):
        lib().eao_set_time(self._h, t)

    def share_noise(self, shared_id: int):
        """Draw Metropolis words from the shared stream shared_id (the
        asynchronous multispin coding of Sec. III)."""
        lib().eao_share_noise(self._h, int(shared_id))
        self.shared = int(shared_id)

    def sweep(self, n: int = 1):
        lib().eao_sweep(self._h, n)

    def half_step(self, half: int, perm=None):
        if perm is None:
            lib().eao_half_step(self._h, half)
        else:
            p = np.ascontiguousarray(perm, dtype=np.int64)
            lib().eao_half_step_order(self._h, half, _ptr(p, ctypes.c_int64))

    def snapshot(self, slot: int):
        if lib().eao_snapshot(self._h, slot) != 0:
            raise IndexError(slot)

    def measure(self) -> Obs:
        ac = np.zeros((2, max(self.n_slots, 0)), dtype=np.int64)
        c4 = np.zeros((3, self.L // 2 + 1), dtype=np.int64)
        o = _Obs()
        o.autocorr = _ptr(ac, ctypes.c_int64) if self.n_slots > 0 else None
        o.c4 = _ptr(c4, ctypes.c_int64)
        lib().eao_measure(self._h, ctypes.byref(o))
        return Obs(int(o.t), np.array(o.unsat[:], dtype=np.int64),
                   np.array(o.mag[:], dtype=np.int64), int(o.overlap), ac, c4)

    def c4_shells(self, n_shells: int | None = None) -> np.ndarray:
        """Full-vector C4 sums by minimum-image squared distance (eq. 3);
        n_shells defaults to (L/2)^2 + 1 (all |r| <= L/2)."""
        n = (self.L // 2) ** 2 + 1 if n_shells is None else int(n_shells)
        out = np.zeros(n, dtype=np.int64)
        lib().eao_c4_shells(self._h, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return out

    def spins(self, r: int) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.int8)
        lib().eao_get_spins(self._h, r, _ptr(out, ctypes.c_int8))
        return out

    def set_spins(self, r: int, S):
        S = np.ascontiguousarray(S, dtype=np.int8)
        assert S.size == self.N
        lib().eao_set_spins(self._h, r, _ptr(S, ctypes.c_int8))

    def bonds(self) -> np.ndarray:
        out = np.zeros(3 * self.N, dtype=np.int8)
        lib().eao_get_bonds(self._h, _ptr(out, ctypes.c_int8))
        return out

    def set_bonds(self, J):
        J = np.ascontiguousarray(J, dtype=np.int8)
        assert J.size == 3 * self.N
        lib().eao_set_bonds(self._h, _ptr(J, ctypes.c_int8))
