"""Pins of the oracle's gamma matrices and hopping term against mathematics.

Each test checks the oracle against something other than itself: algebraic
identities, the closed-form free-field spectrum, gauge covariance, the
point-source stencil and a brute-force sparse matrix.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from gen import fields
from oracle import dirac, evenodd
from oracle.dense import dense
from tests import bruteforce


def test_gamma_algebra():
    g = dirac.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu))
    assert np.allclose(dirac.GAMMA5, np.diag([1, 1, -1, -1]))


def test_gamma_matches_explicit_rows():
    assert np.array_equal(dirac.GAMMA, bruteforce.GAMMA_ROWS)


def match_multiset(a, b):
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    return cost[r, c].max()


def free_momenta(dims):
    lx, ly, lz, lt = dims
    ps = []
    for nx in range(lx):
        for ny in range(ly):
            for nz in range(lz):
                for nt in range(lt):
                    ps.append((2 * np.pi * nx / lx, 2 * np.pi * ny / ly,
                               2 * np.pi * nz / lz, np.pi * (2 * nt + 1) / lt))
    return np.array(ps)


def free_eigenvalues(dims, kappa):
    """lambda_pm(p) = 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), each 6-fold."""
    p = free_momenta(dims)
    c = np.cos(p).sum(1)
    s = np.sqrt((np.sin(p) ** 2).sum(1))
    lp = 1 - 2 * kappa * c + 2j * kappa * s
    lm = 1 - 2 * kappa * c - 2j * kappa * s
    return np.concatenate([np.repeat(lp, 6), np.repeat(lm, 6)])


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (4, 2, 2, 4)])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_free_field_spectrum(dims, csw):
    kappa = 0.11
    u = fields.gauge_field(dims, "unit", 0)
    wc = evenodd.WilsonClover(u, kappa, csw)
    shp = u.shape[:4] + (4, 3)
    m = dense(wc.M, shp)
    ev = np.linalg.eigvals(m)
    assert match_multiset(ev, free_eigenvalues(dims, kappa)) < 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_free_schur_spectrum(dims):
    kappa = 0.11
    u = fields.gauge_field(dims, "unit", 0)
    wc = evenodd.WilsonClover(u, kappa, 1.0)
    v = int(np.prod(dims))
    m = dense(wc.schur, (v // 2, 4, 3))
    ev = np.linalg.eigvals(m)
    p = free_momenta(dims)
    c = np.cos(p).sum(1)
    s = np.sqrt((np.sin(p) ** 2).sum(1))
    lam = np.concatenate([1 - 2 * kappa * c + 2j * kappa * s,
                          1 - 2 * kappa * c - 2j * kappa * s])
    expect = np.repeat(1 - (1 - lam) ** 2, 3)
    assert match_multiset(ev, expect) < 1e-12


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_gamma5_hermiticity(csw):
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "haar", 11)
    wc = evenodd.WilsonClover(u, 0.12, csw)
    phi = fields.gaussian_spinor(dims, 12)
    psi = fields.gaussian_spinor(dims, 13)
    g5 = dirac.gamma5
    lhs = dirac.inner(phi, g5(wc.M(g5(psi))))
    rhs = dirac.inner(wc.M(phi), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)
    # the explicit adjoint agrees too
    assert abs(dirac.inner(phi, wc.Mdag(psi)) - rhs) <= 1e-13 * abs(rhs)


def gauge_rotate(u, g):
    """U'_mu(x) = g(x) U_mu(x) g(x+mu)^dagger."""
    out = np.empty_like(u)
    for mu in range(4):
        gs = dirac.shift(g, mu, +1, antiperiodic_t=False)
        out[..., mu, :, :] = g @ u[..., mu, :, :] @ np.conj(np.swapaxes(gs, -1, -2))
    return out


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_gauge_covariance(csw):
    dims = (4, 4, 2, 4)
    u = fields.gauge_field(dims, "haar", 21)
    g = fields.gauge_transform(dims, 22)
    psi = fields.gaussian_spinor(dims, 23)
    wc = evenodd.WilsonClover(u, 0.13, csw)
    wc2 = evenodd.WilsonClover(gauge_rotate(u, g), 0.13, csw)
    lhs = wc2.M(dirac.colour_mul(g, psi))
    rhs = dirac.colour_mul(g, wc.M(psi))
    assert dirac.norm(lhs - rhs) <= 1e-13 * dirac.norm(rhs)


@pytest.mark.parametrize("y", [(1, 2, 3, 0), (0, 0, 0, 3), (3, 1, 0, 2)])
def test_point_source_stencil(y):
    """For psi = delta_{x,y} chi: (H psi)(y - mu) = (1 - g_mu) U_mu(y - mu) chi and
    (H psi)(y + mu) = (1 + g_mu) U_mu(y)^dagger chi, with -1 across the t boundary."""
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "haar", 31)
    chi = fields.complex_gaussian(fields.rng(32), (4, 3))
    psi = np.zeros(u.shape[:4] + (4, 3), dtype=np.complex128)
    x0, x1, x2, x3 = y
    psi[x3, x2, x1, x0] = chi
    h = dirac.hop(u, psi)
    expect = np.zeros_like(h)
    for mu in range(4):
        c = list(y)
        c[mu] = (c[mu] - 1) % dims[mu]
        sgn = -1.0 if (mu == 3 and y[3] == 0) else 1.0
        lnk = u[c[3], c[2], c[1], c[0], mu]
        expect[c[3], c[2], c[1], c[0]] += sgn * (np.eye(4) - dirac.GAMMA[mu]) @ (chi @ lnk.T)
        c = list(y)
        c[mu] = (c[mu] + 1) % dims[mu]
        sgn = -1.0 if (mu == 3 and y[3] == dims[3] - 1) else 1.0
        lnk = u[x3, x2, x1, x0, mu]
        expect[c[3], c[2], c[1], c[0]] += sgn * (np.eye(4) + dirac.GAMMA[mu]) @ (chi @ lnk.conj())
    assert np.max(np.abs(h - expect)) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 2, 4), (4, 4, 4, 4)])
def test_hop_matches_bruteforce(dims):
    u = fields.gauge_field(dims, "haar", 41)
    psi = fields.gaussian_spinor(dims, 42)
    hm = bruteforce.hopping_matrix(u, dims)
    for dag in (False, True):
        y = dirac.hop(u, psi, dagger=dag).reshape(-1)
        m = hm.conj().T if dag else hm
        ref = m @ psi.reshape(-1)
        assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)


def test_hop_is_antiperiodic_in_t_only():
    """A constant spinor on unit links: H psi = 8 psi in the bulk, but the two
    t-hops across the boundary flip sign, giving 8 - 2*2 = 4 at the t edges."""
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "unit", 0)
    chi = np.zeros((4, 3), dtype=np.complex128)
    chi[0, 0] = 1.0
    psi = np.broadcast_to(chi, u.shape[:4] + (4, 3)).copy()
    h = dirac.hop(u, psi)
    # spatial parts: sum_mu (1-g)+(1+g) = 2 per mu; t part likewise in the bulk
    bulk = h[1, 0, 0, 0]
    edge = h[0, 0, 0, 0]
    assert np.allclose(bulk, 8 * chi)
    # at x3 = 0 the backward t hop flips: (1+g4)(-chi) + (1-g4) chi = -2 g4 chi
    expect = 6 * chi - 2 * dirac.GAMMA[3] @ chi
    assert np.allclose(edge, expect)


def test_hop_at_matches_hop():
    dims = (4, 2, 6, 4)
    u = fields.gauge_field(dims, "haar", 45)
    psi = fields.gaussian_spinor(dims, 46)
    for dag in (False, True):
        h = dirac.hop(u, psi, dagger=dag)
        for site in [(0, 0, 0, 0), (3, 1, 5, 3), (2, 0, 3, 0), (1, 1, 1, 3)]:
            x0, x1, x2, x3 = site
            assert np.max(np.abs(dirac.hop_at(u, psi, site, dag) - h[x3, x2, x1, x0])) < 1e-14
