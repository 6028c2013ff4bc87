"""Site-local SU(3) array expressions in FP64 (oracle; test infrastructure only).

Section 3 of the paper works through the product of arrays of complex 3x3
matrices, U_x = sum_c V_x,a,c W_x,c,b for every x (eq. su3vecmul): 18 x 16
bytes loaded and 9 x 16 stored per element in double precision, 108 complex
multiply-adds, memory-bound.  Section 4 evaluates such element-wise lattice
expressions through QDP++.  These functions are the plain definitions: NumPy
products over the element axis.

Pins (tests/test_oracle_su3.py): explicit triple loops on a few elements;
det(V W) = det V det W; products of SU(3) matrices stay in SU(3); the
paper's byte and flop counts for the element.
"""
from __future__ import annotations

import numpy as np


def mul(v, w):
    """U_x = V_x W_x for arrays (n, 3, 3)."""
    return np.einsum("xac,xcb->xab", v, w)


def dag(v):
    return np.conj(np.swapaxes(v, -1, -2))


def mul_spinor(u, psi):
    """out_x = U_x psi_x on each spin: u (n, 3, 3), psi (n, 4, 3)."""
    return np.einsum("xab,xsb->xsa", u, psi)


def element_bytes(nbytes_complex=16):
    """Bytes moved per element of eq. su3vecmul: two matrices in, one out."""
    return (2 * 9 + 9) * nbytes_complex


def element_madds():
    """Complex multiply-adds per element: 27, i.e. 108 real fused multiply-adds."""
    return 27
