"""Dense matrices of lattice operators on tiny lattices (oracle, test infrastructure).

Column j of the dense matrix is the operator applied to the j-th unit
vector; the index of a full spinor is ((site * 4) + spin) * 3 + colour with
the canonical site order.  Used for brute-force checks (spectra, dense LU
solves, Schur complements) on 2^4 .. 4^4 lattices.
"""
from __future__ import annotations

import numpy as np


def dense(op, shape) -> np.ndarray:
    n = int(np.prod(shape))
    out = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        out[:, j] = op(e.reshape(shape)).reshape(-1)
        e[j] = 0.0
    return out
