"""Brute-force sparse Wilson-clover matrix for tiny lattices (test helper).

Written independently of ``oracle/``: explicit loops over sites and
directions, neighbour coordinates taken modulo the extents, the t-boundary
sign applied to every hop that crosses it, gamma matrices written out as
explicit rows (chiral basis).  Used to pin the oracle's stencil, even-odd
reduction and solvers with a direct sparse solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Explicit rows of the chiral-basis gamma matrices (mu = 0..3 <-> x, y, z, t).
I = 1j
GAMMA_ROWS = np.array([
    [[0, 0, 0, -I], [0, 0, -I, 0], [0, I, 0, 0], [I, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, -I, 0], [0, 0, 0, I], [I, 0, 0, 0], [0, -I, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)


def site_index(c, dims):
    x0, x1, x2, x3 = c
    lx, ly, lz, lt = dims
    return ((x3 * lz + x2) * ly + x1) * lx + x0


def coords(i, dims):
    lx, ly, lz, lt = dims
    x0 = i % lx
    i //= lx
    x1 = i % ly
    i //= ly
    x2 = i % lz
    x3 = i // lz
    return [x0, x1, x2, x3]


def hopping_matrix(u, dims, antiperiodic_t=True):
    """Sparse H (12V x 12V), index (site*4 + spin)*3 + colour."""
    v = int(np.prod(dims))
    ug = u.reshape(v, 4, 3, 3)
    one = np.eye(4)
    rows, cols, vals = [], [], []
    for i in range(v):
        c = coords(i, dims)
        for mu in range(4):
            # forward neighbour
            cf = list(c)
            cf[mu] += 1
            sf = 1.0
            if cf[mu] == dims[mu]:
                cf[mu] = 0
                if mu == 3 and antiperiodic_t:
                    sf = -1.0
            jf = site_index(cf, dims)
            blk_f = sf * np.kron(one - GAMMA_ROWS[mu], ug[i, mu])
            # backward neighbour
            cb = list(c)
            cb[mu] -= 1
            sb = 1.0
            if cb[mu] < 0:
                cb[mu] = dims[mu] - 1
                if mu == 3 and antiperiodic_t:
                    sb = -1.0
            jb = site_index(cb, dims)
            blk_b = sb * np.kron(one + GAMMA_ROWS[mu], ug[jb, mu].conj().T)
            for j, blk in ((jf, blk_f), (jb, blk_b)):
                for a in range(12):
                    for b in range(12):
                        if blk[a, b] != 0:
                            rows.append(12 * i + a)
                            cols.append(12 * j + b)
                            vals.append(blk[a, b])
    # duplicates (extent-2 directions) are summed by the COO -> CSR conversion
    return sp.coo_matrix((vals, (rows, cols)), shape=(12 * v, 12 * v)).tocsr()


def clover_block_matrix(a_sites):
    """Block-diagonal sparse matrix from per-site 12x12 clover blocks."""
    return sp.block_diag(list(a_sites), format="csr")


def parity_of_sites(dims):
    v = int(np.prod(dims))
    return np.array([sum(coords(i, dims)) % 2 for i in range(v)])
