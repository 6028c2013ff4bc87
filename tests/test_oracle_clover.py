"""Pins of the oracle's clover term: closed forms and invariants."""
import numpy as np
import pytest

from gen import fields
from oracle import clover, dirac, evenodd
from tests.test_oracle_dirac import gauge_rotate


def abelian_field(dims, mu, nu, n_flux):
    """Constant abelian field in the mu-nu plane, charges q = (1, -1, 0).

    Flux theta = 2 pi n / (L_mu L_nu) per plaquette: U_nu(x) = exp(i q theta x_mu),
    U_mu(x) = exp(-i q theta L_mu x_nu) on the last x_mu slice, 1 elsewhere.
    """
    lt, lz, ly, lx = fields.lattice_shape(dims)
    theta = 2 * np.pi * n_flux / (dims[mu] * dims[nu])
    q = np.array([1.0, -1.0, 0.0])
    u = fields.gauge_field(dims, "unit", 0).copy()
    for x3 in range(lt):
        for x2 in range(lz):
            for x1 in range(ly):
                for x0 in range(lx):
                    c = (x0, x1, x2, x3)
                    u[x3, x2, x1, x0, nu] = np.diag(np.exp(1j * q * theta * c[mu]))
                    if c[mu] == dims[mu] - 1:
                        u[x3, x2, x1, x0, mu] = np.diag(
                            np.exp(-1j * q * theta * dims[mu] * c[nu]))
    return u, theta, q


@pytest.mark.parametrize("plane", [(0, 1), (1, 3), (0, 3), (2, 3)])
def test_abelian_field_strength_closed_form(plane):
    dims = (4, 4, 4, 6)
    mu, nu = plane
    u, theta, q = abelian_field(dims, mu, nu, 1)
    for a in range(4):
        for b in range(a + 1, 4):
            f = clover.field_strength(u, a, b)
            if (a, b) == (mu, nu):
                expect = np.diag(np.sin(q * theta))
            else:
                expect = np.zeros((3, 3))
            assert np.max(np.abs(f - expect)) < 1e-14


def test_unit_links_clover_is_identity():
    dims = (4, 2, 2, 4)
    a = clover.clover_matrix(fields.gauge_field(dims, "unit", 0), 0.135, 1.0)
    assert np.max(np.abs(a - np.eye(12))) < 1e-15


def test_clover_hermitian_chiral_blocks_and_inverse():
    dims = (4, 4, 2, 4)
    u = fields.gauge_field(dims, "haar", 51)
    a = clover.clover_matrix(u, 0.135, 1.0)
    assert np.max(np.abs(a - np.conj(np.swapaxes(a, -1, -2)))) < 1e-15
    g5 = np.kron(dirac.GAMMA5, np.eye(3))
    assert np.max(np.abs(a @ g5 - g5 @ a)) < 1e-15
    # chirality blocks: spins {0,1} and {2,3} do not mix
    assert np.max(np.abs(a[..., :6, 6:])) < 1e-15
    ai = clover.invert_site_matrix(a)
    assert np.max(np.abs(a @ ai - np.eye(12))) < 1e-13


def test_field_strength_gauge_covariant():
    dims = (4, 4, 2, 4)
    u = fields.gauge_field(dims, "haar", 61)
    g = fields.gauge_transform(dims, 62)
    ur = gauge_rotate(u, g)
    for mu, nu in [(0, 1), (0, 3), (2, 3)]:
        f = clover.field_strength(u, mu, nu)
        fr = clover.field_strength(ur, mu, nu)
        assert np.max(np.abs(fr - g @ f @ np.conj(np.swapaxes(g, -1, -2)))) < 1e-14


def test_field_strength_traceless_hermitian_antisymmetric():
    dims = (2, 4, 2, 4)
    u = fields.gauge_field(dims, "smooth", 71)
    f01 = clover.field_strength(u, 0, 1)
    assert np.max(np.abs(np.trace(f01, axis1=-2, axis2=-1))) < 1e-15
    assert np.max(np.abs(f01 - np.conj(np.swapaxes(f01, -1, -2)))) < 1e-15
    # orientation: F_{nu mu} = -F_{mu nu}
    assert np.max(np.abs(clover.field_strength(u, 1, 0) + f01)) < 1e-15


def test_weak_abelian_field_matches_continuum():
    """On a weak constant field, (Q - Q^dag)/(8i) ~ q theta: the lattice field
    strength tends to the continuum one (sin x -> x)."""
    dims = (16, 16, 2, 2)
    u, theta, q = abelian_field(dims, 0, 1, 1)
    f = clover.field_strength(u, 0, 1)
    assert np.allclose(np.diagonal(f[0, 0, 0, 0]).real, q * theta, atol=theta ** 3)


def test_clover_sigma_f_sign_in_abelian_field():
    """In the abelian field, A restricted to colour 0 is 1 - csw kappa sigma_{01} sin(theta);
    sigma_{01} = diag(-1, 1, -1, 1) in the chiral basis, so spin 0 gets
    1 + csw kappa sin(theta) and spin 1 gets 1 - csw kappa sin(theta)."""
    dims = (4, 4, 2, 2)
    u, theta, q = abelian_field(dims, 0, 1, 1)
    kappa, csw = 0.125, 1.0
    a = clover.clover_matrix(u, kappa, csw)[0, 0, 0, 0]
    s01 = 0.5j * (dirac.GAMMA[0] @ dirac.GAMMA[1] - dirac.GAMMA[1] @ dirac.GAMMA[0])
    assert np.allclose(s01, np.diag([-1, 1, -1, 1]))
    # index 3*spin + colour; colour 0 has charge +1
    assert abs(a[0, 0] - (1 + csw * kappa * np.sin(theta))) < 1e-15
    assert abs(a[3, 3] - (1 - csw * kappa * np.sin(theta))) < 1e-15


def test_clover_operator_gamma5_hermitian_smooth():
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "smooth", 81)
    wc = evenodd.WilsonClover(u, 0.135, 1.0)
    phi = fields.gaussian_spinor(dims, 82)
    psi = fields.gaussian_spinor(dims, 83)
    g5 = dirac.gamma5
    lhs = dirac.inner(phi, g5(wc.M(g5(psi))))
    rhs = dirac.inner(wc.M(phi), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


def test_clover_cancels_pauli_term_at_csw_one():
    """Pin of the clover sign and normalisation from the O(a) argument.

    The Wilson term -(1/2) sum_mu Delta_mu equals -(1/2)(gamma.nabla)^2 plus a
    spin term +(1/2) sum_{mu<nu} sigma F (for smooth fields), which the clover
    term -csw kappa sum sigma F removes at csw = 1.  On a smooth plane wave in a
    weak constant abelian field, M(csw) is compared with
    (1 - 8 kappa) - kappa (gamma.nabla)^2 + 2 kappa gamma.nabla built from the
    symmetric covariant difference nabla; the residual, quadratic in csw, has
    its minimum near csw = 1 (away from the gauge seam of the field).
    """
    dims = (32, 32, 2, 2)
    u, theta, q = abelian_field(dims, 0, 1, 1)
    kappa = 0.125
    lt, lz, ly, lx = fields.lattice_shape(dims)
    x3, x2, x1, x0 = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                                 np.arange(lx), indexing="ij")
    p = 2 * np.pi / 32
    chi = fields.complex_gaussian(fields.rng(5), (4, 3))
    f = np.exp(1j * p * (x0 + x1))[..., None, None] * chi

    def nabla(psi, mu):
        um = u[..., mu, :, :]
        return 0.5 * (dirac.colour_mul(um, dirac.shift(psi, mu, 1, False))
                      - dirac.shift(dirac.colour_mul_dag(um, psi), mu, -1, False))

    def gnabla(psi):
        return sum(dirac.spin_mul(dirac.GAMMA[mu], nabla(psi, mu)) for mu in range(4))

    ref = (1 - 8 * kappa) * f - kappa * gnabla(gnabla(f)) + 2 * kappa * gnabla(f)
    away = (x0 >= 3) & (x0 <= lx - 4)
    d2 = {}
    for c in (1.0, 0.0, -1.0):
        wc = evenodd.WilsonClover(u, kappa, c, antiperiodic_t=False)
        d2[c] = float(np.linalg.norm((wc.M(f) - ref)[away]) ** 2)
    curv = (d2[1.0] + d2[-1.0] - 2 * d2[0.0]) / 2
    slope = (d2[1.0] - d2[-1.0]) / 4
    c_best = -slope / curv
    assert 0.8 < c_best < 1.3
    assert d2[1.0] < 0.2 * d2[0.0] < d2[-1.0]
