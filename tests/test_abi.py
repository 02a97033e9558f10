"""Host-side checks of the C ABI that run without a GPU: the library loads,
exports every function include/ea.h declares, and its host logic (argument
checks, thresholds, footprints) behaves as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "ea.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ea_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ealib():
    from paper_1411_5512_amd import abi
    if not os.path.exists(abi.LIB_PATH):
        pytest.skip("libea.so not built")
    return abi


def test_every_declared_symbol_is_exported(ealib):
    names = _declared_functions()
    assert len(names) >= 17
    lib = ctypes.CDLL(ealib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    # the binding declares exactly the header's functions
    assert sorted(ealib.exported_names()) == names


def test_thresholds_match_oracle(ealib, oracle_mod):
    import paper_1411_5512_amd as ea
    from test_oracle_rng import EXACT_THRESHOLDS
    for T, want in EXACT_THRESHOLDS.items():  # eq. (9) floor rule, worked out in decimals
        assert tuple(int(v) for v in ea.thresholds(T)) == want, T
    for T in [0.0, 0.3, 0.5, 0.6, 0.7, 0.8, 1.0, 1.2, 4.5, 1e300]:
        assert list(ea.thresholds(T)) == list(oracle_mod.thresholds(T))
    with pytest.raises(ea.EAError):
        ea.thresholds(-1.0)
    with pytest.raises(ea.EAError):
        ea.thresholds(float("nan"))


def test_footprint_and_bad_arguments(ealib):
    import paper_1411_5512_amd as ea
    # densest packing (32 sites per word where the row allows): 2 replicas x N
    # bits of spins + 3N bits of couplings (plus padding); W sites per 32-bit
    # word cost 32 / W times that.  A packing that can run as slabs (a colour
    # plane of L rw <= 1024 words) adds the exchange area: 3 slots x 2
    # replicas x 2 colours of 64-bit entries per packed word.
    for L, rw, W in ((16, 1, 8), (64, 1, 32), (128, 2, 32), (64, 8, 4), (96, 4, 12), (256, 8, 16)):
        fp = ea.footprint(L, words_per_row=rw)
        dense = 5 * L ** 3 // 8 * 32 // W
        xbuf = 12 * 8 * L * L * rw if L * rw <= 1024 else 0
        assert dense + xbuf <= fp < dense + xbuf + 4096 + 8 * 2000, (L, rw)
        assert ea.footprint(L) >= ea.footprint(L, words_per_row={16: 1, 64: 1, 128: 2, 96: 2, 256: 4}[L])
    assert ea.footprint(64, 3, words_per_row=1) - ea.footprint(64, 0, words_per_row=1) >= 3 * 2 * 64 ** 3 // 8
    for L, rw in ((64, 3), (64, 16), (96, 5), (16, 0 - 1)):  # not whole 4-site blocks, or W < 4
        with pytest.raises(ea.EAError):
            ea.footprint(L, words_per_row=rw)
    for L in (0, 4, 12, 260, 264, -8):
        with pytest.raises(ea.EAError):
            ea.footprint(L)
    with pytest.raises(ea.EAError):
        ea.footprint(16, 65)
    for args in [(12, 0.5, 0.8), (16, -0.1, 0.8), (16, 1.5, 0.8), (16, 0.5, -0.1),
                 (16, 0.5, float("inf")), (16, float("nan"), 0.8)]:
        h = ctypes.c_void_p()
        st = ealib.lib().ea_create(args[0], args[1], args[2], 1, ctypes.byref(h))
        assert st == ealib.EA_ERR_ARG and not h.value
        assert ealib.lib().ea_last_error()


def test_msc_footprint_and_bad_arguments(ealib):
    """Host logic of the multispin-coded batch: device bytes (bits of every
    sample's spins, couplings and snapshots, plus counters) and the packing
    rules (32 / M slabs of even depth, word sets of 32 samples)."""
    import paper_1411_5512_amd as ea
    for L, B, slots in ((128, 64, 0), (128, 32, 2), (16, 8, 1), (64, 1, 0), (24, 16, 3), (8, 256, 0)):
        fp = ea.Msc.footprint(L, B, slots)
        # words per plane, all word sets: 32 samples per word; fewer samples fill
        # the 32 bits with 32 / B slabs of L B / 32 planes each
        words = (B // 32 if B >= 32 else 1) * (L // 2) * L * (L if B >= 32 else L * B // 32)
        dense = 4 * words * (4 + 6 + 4 * slots + 2)   # spins, couplings, snapshots, overlap words
        counters = 8 * (5 + 2 * 64 + 3 * (L // 2 + 1)) * (max(B, 32) // 32) * 32
        assert dense + counters <= fp < dense + counters + 5 * 256 + 256, (L, B, slots)
    for L, B in ((16, 3), (16, 0), (16, 48), (16, 288), (24, 1), (40, 2), (8, 4), (12, 32), (264, 32)):
        with pytest.raises(ea.EAError):
            ea.Msc.footprint(L, B)
    with pytest.raises(ea.EAError):
        ea.Msc.footprint(16, 32, 65)


def test_debug_mode_flags(ealib):
    """ea_set_debug / ea_get_debug: any combination of the three flags with a
    seed is kept process-wide; unknown bits are rejected and leave the mode
    unchanged; 0 switches it off (host only: no launch)."""
    import paper_1411_5512_amd as ea
    try:
        assert ea.get_debug() == (0, 0)
        ea.set_debug(ea.DEBUG_REVERSE | ea.DEBUG_POISON, 0xDEADBEEF)
        assert ea.get_debug() == (5, 0xDEADBEEF)
        with pytest.raises(ea.EAError):
            ea.set_debug(8, 1)
        assert ea.get_debug() == (5, 0xDEADBEEF)
        ea.set_debug(ea.DEBUG_ROTATE, 3)
        assert ea.get_debug() == (2, 3)
    finally:
        ea.set_debug(0, 0)
    assert ea.get_debug() == (0, 0)


def test_shell_route_setting(ealib):
    """ea_set_shell_route / ea_get_shell_route: the three routes are kept
    process-wide, another value is rejected and leaves the route unchanged
    (host only: no launch)."""
    import paper_1411_5512_amd as ea
    try:
        assert ea.get_shell_route() == ea.SHELLS_AUTO
        ea.set_shell_route(ea.SHELLS_FFT)
        assert ea.get_shell_route() == ea.SHELLS_FFT
        for bad in (-1, 3):
            with pytest.raises(ea.EAError):
                ea.set_shell_route(bad)
        assert ea.get_shell_route() == ea.SHELLS_FFT
        ea.set_shell_route(ea.SHELLS_DIRECT)
        assert ea.get_shell_route() == ea.SHELLS_DIRECT
    finally:
        ea.set_shell_route(ea.SHELLS_AUTO)
    assert ea.get_shell_route() == ea.SHELLS_AUTO
