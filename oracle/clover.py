"""Clover term A of the Wilson-clover operator (FP64 oracle, test infrastructure).

Paper: section 3 names "Clover fermions" as one of the two operator
formulations considered; it does not define the term.  Reading used here
(tree-level improved Sheikholeslami-Wohlert term in the kappa normalisation):

    M = A - kappa H,   A(x) = 1 - c_sw kappa sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
    sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
    F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dagger) / (8i), minus its trace / 3,

with Q_{mu nu}(x) the sum of the four plaquette leaves at x in the mu-nu
plane, each ordered mu then nu (counter-clockwise), gauge links periodic.
F is Hermitian and traceless; A is Hermitian and commutes with gamma_5.

Pins (CPU tests): unit links give A = 1; a constant abelian field with flux
theta per plaquette gives F = diag(sin(q theta)) exactly; Hermiticity;
[A, gamma_5] = 0; gauge covariance of F; A A^{-1} = 1.  The overall sign of
the clover term relative to F follows from the derivation (Wilson term
-(a/2) D^2 contains +(a/4) sigma F, which c_sw = 1 cancels); no value
printed in the paper fixes it.

A^{-1} is the full 12x12 LU inverse per site (no use of the chiral block
structure).
"""
from __future__ import annotations

import numpy as np

from .dirac import GAMMA, shift


def _sigma_munu() -> np.ndarray:
    s = np.zeros((4, 4, 4, 4), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            s[mu, nu] = 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
    return s


SIGMA_MUNU = _sigma_munu()


def _at(u_mu: np.ndarray, offsets) -> np.ndarray:
    """u_mu(x + sum_k step_k * dir_k) for a list of (dir, step), periodic."""
    out = u_mu
    for d, step in offsets:
        out = shift(out, d, step, antiperiodic_t=False)
    return out


def _dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def clover_leaves(u: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): the four plaquettes at x in the mu-nu plane, mu -> nu ordered."""
    um = u[..., mu, :, :]
    un = u[..., nu, :, :]
    # leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
    q = um @ _at(un, [(mu, 1)]) @ _dag(_at(um, [(nu, 1)])) @ _dag(un)
    # leaf 2: x -> x-nu -> x-nu+mu -> x+mu -> x
    q = q + (_dag(_at(un, [(nu, -1)])) @ _at(um, [(nu, -1)])
             @ _at(un, [(nu, -1), (mu, 1)]) @ _dag(um))
    # leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + (_dag(_at(um, [(mu, -1)])) @ _dag(_at(un, [(mu, -1), (nu, -1)]))
             @ _at(um, [(mu, -1), (nu, -1)]) @ _at(un, [(nu, -1)]))
    # leaf 4: x -> x+nu -> x+nu-mu -> x-mu -> x
    q = q + (un @ _dag(_at(um, [(mu, -1), (nu, 1)])) @ _dag(_at(un, [(mu, -1)]))
             @ _at(um, [(mu, -1)]))
    return q


def field_strength(u: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Hermitian traceless F_{mu nu}(x) = (Q - Q^dagger)/(8i) - tr/3."""
    q = clover_leaves(u, mu, nu)
    f = (q - _dag(q)) / 8j
    tr = np.trace(f, axis1=-2, axis2=-1)
    return f - (tr / 3.0)[..., None, None] * np.eye(3)


def clover_matrix(u: np.ndarray, kappa: float, csw: float) -> np.ndarray:
    """A(x) as a 12x12 matrix per site, row/column index 3*spin + colour."""
    lat = u.shape[:4]
    a = np.zeros(lat + (12, 12), dtype=np.complex128)
    a[...] = np.eye(12)
    if csw == 0.0:
        return a
    for mu in range(4):
        for nu in range(mu + 1, 4):
            f = field_strength(u, mu, nu)
            a -= csw * kappa * np.einsum("st,...ab->...satb", SIGMA_MUNU[mu, nu],
                                         f).reshape(lat + (12, 12))
    return a


def apply_site_matrix(m: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """y(x) = m(x) psi(x) with m a 12x12 matrix on (spin, colour)."""
    shp = psi.shape
    v = psi.reshape(shp[:-2] + (12,))
    return np.einsum("...ij,...j->...i", m, v).reshape(shp)


def invert_site_matrix(m: np.ndarray) -> np.ndarray:
    """Per-site 12x12 inverse (LAPACK LU with partial pivoting)."""
    return np.linalg.inv(m)
