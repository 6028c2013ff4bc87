"""Gamma matrices and the Wilson hopping term (FP64 oracle, test infrastructure).

Paper: section 3 states the problem for Wilson or clover fermions, whose
matrix M is sparse, complex and not Hermitian; section 5 notes that the
matrix-vector product is the dominant cost.  The paper does not define the
operator.  Readings used here (each pinned by a CPU test):

* Euclidean Hermitian gamma matrices in the chiral basis, built from the Pauli
  matrices: gamma_k = [[0, -i s_k], [i s_k, 0]] for k = 1,2,3 (mu = 0,1,2),
  gamma_4 = [[0, 1], [1, 0]] (mu = 3), gamma_5 = gamma_1 gamma_2 gamma_3
  gamma_4 = diag(1, 1, -1, -1).
* Hopping term with Wilson parameter r = 1 and the kappa normalisation:
  (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
                       + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)],
  M_W = 1 - kappa H.
* Boundary conditions: gauge links periodic; fermion hops periodic in x, y, z
  and antiperiodic in t (a hop across the t boundary carries a factor -1).
  On an extent-2 direction both hops land on the same neighbour and add.

Arrays: full-lattice fields have leading axes (Lt, Lz, Ly, Lx); a spinor has
trailing axes (spin 4, colour 3); a gauge field has trailing (mu 4, 3, 3).
"""
from __future__ import annotations

import numpy as np

SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)


def _gammas() -> np.ndarray:
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    z = np.zeros((2, 2), dtype=np.complex128)
    for k in range(3):
        g[k] = np.block([[z, -1j * SIGMA[k]], [1j * SIGMA[k], z]])
    g[3] = np.block([[z, np.eye(2)], [np.eye(2), z]])
    return g


GAMMA = _gammas()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)

# Lattice axis holding direction mu in a (Lt, Lz, Ly, Lx, ...) array.
AXIS = (3, 2, 1, 0)


def shift(field: np.ndarray, mu: int, step: int, antiperiodic_t: bool) -> np.ndarray:
    """Return f with f(x) = field(x + step*mu_hat), step = +1 or -1.

    With antiperiodic_t and mu = 3 the values that wrapped around the t
    boundary are negated (fermion boundary condition).  Gauge fields are
    shifted with antiperiodic_t = False.
    """
    ax = AXIS[mu]
    out = np.roll(field, -step, axis=ax)
    if antiperiodic_t and mu == 3:
        idx = [slice(None)] * out.ndim
        idx[ax] = -1 if step > 0 else 0
        out[tuple(idx)] *= -1.0
    return out


def colour_mul(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)_{s,a} = sum_b U_{ab} psi_{s,b}, site by site."""
    return np.einsum("...ab,...sb->...sa", u, psi)


def colour_mul_dag(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U^dagger psi)_{s,a} = sum_b conj(U_{ba}) psi_{s,b}."""
    return np.einsum("...ba,...sb->...sa", u.conj(), psi)


def spin_mul(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(G psi)_{s,a} = sum_t G_{st} psi_{t,a} for a 4x4 spin matrix G."""
    return np.einsum("st,...ta->...sa", g, psi)


def hop(u: np.ndarray, psi: np.ndarray, dagger: bool = False,
        antiperiodic_t: bool = True) -> np.ndarray:
    """Hopping term H psi (or H^dagger psi) on the full lattice.

    H^dagger swaps the projectors: (1 + gamma_mu) on the forward hop and
    (1 - gamma_mu) on the backward hop.
    """
    out = np.zeros_like(psi)
    sgn = -1.0 if dagger else 1.0
    for mu in range(4):
        u_mu = u[..., mu, :, :]
        fwd = colour_mul(u_mu, shift(psi, mu, +1, antiperiodic_t))
        bwd = shift(colour_mul_dag(u_mu, psi), mu, -1, antiperiodic_t)
        out += spin_mul(ONE4 - sgn * GAMMA[mu], fwd)
        out += spin_mul(ONE4 + sgn * GAMMA[mu], bwd)
    return out


def wilson(u: np.ndarray, psi: np.ndarray, kappa: float, dagger: bool = False,
           antiperiodic_t: bool = True) -> np.ndarray:
    """M_W psi = psi - kappa H psi (dagger: psi - kappa H^dagger psi)."""
    return psi - kappa * hop(u, psi, dagger, antiperiodic_t)


def gamma5(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, psi)


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a_i) b_i."""
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def norm(a: np.ndarray) -> float:
    return float(np.linalg.norm(a.reshape(-1)))


def hop_at(u: np.ndarray, psi: np.ndarray, site, dagger: bool = False,
           antiperiodic_t: bool = True) -> np.ndarray:
    """(H psi)(x) at the single site x = (x0, x1, x2, x3), from its eight
    neighbours; the same definition as hop(), evaluated one site at a time so
    that outputs of very large lattices can be sampled."""
    lt, lz, ly, lx = psi.shape[:4]
    ext = (lx, ly, lz, lt)
    x = list(site)
    sgn = -1.0 if dagger else 1.0
    out = np.zeros((4, 3), dtype=np.complex128)
    for mu in range(4):
        f = list(x)
        f[mu] = (x[mu] + 1) % ext[mu]
        b = list(x)
        b[mu] = (x[mu] - 1) % ext[mu]
        bc_f = -1.0 if (antiperiodic_t and mu == 3 and x[3] == ext[3] - 1) else 1.0
        bc_b = -1.0 if (antiperiodic_t and mu == 3 and x[3] == 0) else 1.0
        u_f = u[x[3], x[2], x[1], x[0], mu]
        u_b = u[b[3], b[2], b[1], b[0], mu]
        chi_f = bc_f * (psi[f[3], f[2], f[1], f[0]] @ u_f.T)
        chi_b = bc_b * (psi[b[3], b[2], b[1], b[0]] @ u_b.conj())
        out += (ONE4 - sgn * GAMMA[mu]) @ chi_f
        out += (ONE4 + sgn * GAMMA[mu]) @ chi_b
    return out
