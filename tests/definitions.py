"""Observables computed straight from their definitions on int8 +-1 arrays
in canonical order (s = x + L (y + L z), couplings J[3 s + d] to the +x, +y,
+z neighbour), for checks at sizes where the oracle's full measurement is too
slow.  Independent of both the oracle and the library."""
import numpy as np


def unsat_count(S, J, L):
    """Unsatisfied bonds (J S_i S_j = -1) of one replica; its energy (eq. 1)
    is 2 n_unsat - 3 N."""
    s = S.reshape(L, L, L).astype(np.int32)  # [z][y][x]
    j = J.reshape(L, L, L, 3).astype(np.int32)
    return sum(int(np.count_nonzero(j[..., d] * s * np.roll(s, -1, axis=ax) < 0))
               for d, ax in enumerate((2, 1, 0)))


def axis_c4(q, L):
    """sum_x q(x) q(x + r e_d), r = 0..L/2, along x, y, z (eq. 3 before the
    division by N), by FFT along each axis."""
    g = q.reshape(L, L, L).astype(np.float64)
    out = np.zeros((3, L // 2 + 1), dtype=np.int64)
    for d, ax in enumerate((2, 1, 0)):
        c = np.fft.irfft(np.abs(np.fft.rfft(g, axis=ax)) ** 2, n=L, axis=ax)
        other = tuple(a for a in range(3) if a != ax)
        out[d] = np.rint(c.sum(axis=other)[: L // 2 + 1]).astype(np.int64)
    return out
