"""Even-odd (Schur complement) reduction of M = A - kappa H (FP64 oracle, test infrastructure).

Paper: section 5 describes CG on the Schur complement equation of the
even-odd decomposition of the Wilson operator, whose application needs two
sweeps of the lattice (next-to-nearest neighbour coupling).  The paper does
not write the reduction down.  Reading used here:

    parity pi(x) = (x0 + x1 + x2 + x3) mod 2, even = 0;
    M = [[A_ee, -kappa H_eo], [-kappa H_oe, A_oo]];
    Schur operator  Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe   (acts on even sites),
    source          bhat_e = b_e + kappa H_eo A_oo^{-1} b_o,
    reconstruction  x_o = A_oo^{-1} (b_o + kappa H_oe x_e).

This Mhat is gamma_5-Hermitian (gamma_5 Mhat gamma_5 = Mhat^dagger), which
CG on the normal equations relies on.  Mhat^dagger is formed from H^dagger
directly: A_ee - kappa^2 (H^dagger)_eo A_oo^{-1} (H^dagger)_oe.

Half-lattice fields are arrays (V/2, 4, 3) listing the sites of one parity
in increasing full-lattice index order.  The hopping blocks are taken from
the full-lattice H applied to a field that is zero on the other parity.

Pins (CPU tests): M (x_e, x_o) = b after a Schur solve; the dense Schur
complement built from the dense M; the free-field Schur spectrum.
"""
from __future__ import annotations

import numpy as np

from . import clover as _clover
from . import dirac as _dirac

EVEN, ODD = 0, 1


def odd_mask(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    x3, x2, x1, x0 = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                                 np.arange(lx), indexing="ij")
    return ((x0 + x1 + x2 + x3) % 2) == 1


def lattice_shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


def split(full: np.ndarray, dims) -> tuple[np.ndarray, np.ndarray]:
    """Full-lattice field (Lt,Lz,Ly,Lx,...) -> (even, odd) half-lattice fields."""
    m = odd_mask(dims).reshape(-1)
    flat = full.reshape((m.size,) + full.shape[4:])
    return flat[~m].copy(), flat[m].copy()


def join(even: np.ndarray | None, odd: np.ndarray | None, dims) -> np.ndarray:
    """(even, odd) half-lattice fields -> full-lattice field; None means zero."""
    m = odd_mask(dims).reshape(-1)
    tail = (even if even is not None else odd).shape[1:]
    out = np.zeros((m.size,) + tail, dtype=np.complex128)
    if even is not None:
        out[~m] = even
    if odd is not None:
        out[m] = odd
    return out.reshape(lattice_shape(dims) + tail)


class WilsonClover:
    """The Wilson-clover operator M = A - kappa H on one gauge field.

    csw = 0 gives the plain Wilson operator (A = 1).
    """

    def __init__(self, u: np.ndarray, kappa: float, csw: float = 0.0,
                 antiperiodic_t: bool = True):
        self.u = u
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.apt = antiperiodic_t
        lt, lz, ly, lx = u.shape[:4]
        self.dims = (lx, ly, lz, lt)
        self.a = _clover.clover_matrix(u, kappa, csw)
        self.ainv = _clover.invert_site_matrix(self.a)
        ae, ao = split(self.a, self.dims)
        aie, aio = split(self.ainv, self.dims)
        self.a_half = (ae, ao)
        self.ainv_half = (aie, aio)

    # -- full lattice -------------------------------------------------
    def hop(self, psi, dagger=False):
        return _dirac.hop(self.u, psi, dagger, self.apt)

    def clover(self, psi):
        return _clover.apply_site_matrix(self.a, psi)

    def M(self, psi):
        return self.clover(psi) - self.kappa * self.hop(psi)

    def Mdag(self, psi):
        return self.clover(psi) - self.kappa * self.hop(psi, dagger=True)

    # -- half lattice blocks -----------------------------------------
    def hop_block(self, psi_half, out_parity: int, dagger=False):
        """H_eo (out_parity EVEN, input odd) or H_oe (out_parity ODD, input even)."""
        if out_parity == EVEN:
            full = join(None, psi_half, self.dims)
        else:
            full = join(psi_half, None, self.dims)
        y = self.hop(full, dagger)
        return split(y, self.dims)[out_parity]

    def clover_half(self, psi_half, parity: int, inverse=False):
        m = (self.ainv_half if inverse else self.a_half)[parity]
        return _clover.apply_site_matrix(m, psi_half)

    def schur(self, x_e, dagger=False):
        """Mhat x_e (or Mhat^dagger x_e)."""
        t = self.hop_block(x_e, ODD, dagger)
        t = self.clover_half(t, ODD, inverse=True)
        y = self.hop_block(t, EVEN, dagger)
        return self.clover_half(x_e, EVEN) - self.kappa ** 2 * y

    def prepare_source(self, b_full):
        """bhat_e = b_e + kappa H_eo A_oo^{-1} b_o."""
        b_e, b_o = split(b_full, self.dims)
        t = self.clover_half(b_o, ODD, inverse=True)
        return b_e + self.kappa * self.hop_block(t, EVEN)

    def reconstruct(self, x_e, b_full):
        """Full solution from x_e: x_o = A_oo^{-1} (b_o + kappa H_oe x_e)."""
        _, b_o = split(b_full, self.dims)
        x_o = self.clover_half(b_o + self.kappa * self.hop_block(x_e, ODD), ODD,
                               inverse=True)
        return join(x_e, x_o, self.dims)
