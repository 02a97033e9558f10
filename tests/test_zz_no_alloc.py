"""The allocation-free variant of the full-vector C4 (ea_c4_shells_into,
called through the C ABI): its device results equal ea_c4_shells' on two
calls in a row, the second with a smaller lattice and fewer shells, so that
the shared scratch array is reused with less data than the first call left."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _into(ea, sim, n_shells, torch):
    out = torch.full((n_shells,), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    st = ea.abi.lib().ea_c4_shells_into(sim._h, int(n_shells), ctypes.c_void_p(out.data_ptr()))
    ea.abi.check(st)
    sim.sync()
    return out.cpu().numpy()


def test_no_alloc_shells_equal_the_allocating_call(ea_gpu):
    import torch
    cases = [(128, 0.5, 0.7, 3 * 64 * 64 + 1, 40), (48, 0.3, 0.9, 24 * 24 + 1, 25)]
    for L, p, T, n_shells, sweeps in cases:
        _say(f"no-alloc shells L={L} n_shells={n_shells}")
        s = ea_gpu.Sim(L, p, T, seed=31, sample=1)
        s.sweep(sweeps)
        got = _into(ea_gpu, s, n_shells, torch)
        want = s.c4_shells(n_shells)
        assert got.shape == want.shape
        assert np.array_equal(got, want), (L, np.flatnonzero(got != want)[:8])
        assert got[0] == L ** 3
        s.close()


def test_no_alloc_shells_rejects_beyond_the_scratch(ea_gpu):
    import torch
    s = ea_gpu.Sim(136, 0.5, 0.8, seed=1)
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    st = ea_gpu.abi.lib().ea_c4_shells_into(s._h, 8, ctypes.c_void_p(out.data_ptr()))
    assert st == ea_gpu.abi.EA_ERR_ARG
    s.close()
    s = ea_gpu.Sim(16, 0.5, 0.8, seed=1)
    for n in (0, 3 * 8 * 8 + 2):
        assert ea_gpu.abi.lib().ea_c4_shells_into(s._h, n, ctypes.c_void_p(out.data_ptr())) == ea_gpu.abi.EA_ERR_ARG
    s.close()
