"""Pins of the SU(3) array-expression oracle (oracle/su3.py)."""
import numpy as np

from gen import fields
from oracle import su3


def test_product_matches_explicit_loops():
    rng = fields.rng(601)
    v = fields.complex_gaussian(rng, (5, 3, 3))
    w = fields.complex_gaussian(rng, (5, 3, 3))
    got = su3.mul(v, w)
    for x in range(5):
        for a in range(3):
            for b in range(3):
                ref = sum(v[x, a, c] * w[x, c, b] for c in range(3))
                assert abs(got[x, a, b] - ref) <= 1e-14


def test_determinant_and_group_closure():
    rng = fields.rng(602)
    v = fields.complex_gaussian(rng, (7, 3, 3))
    w = fields.complex_gaussian(rng, (7, 3, 3))
    assert np.allclose(np.linalg.det(su3.mul(v, w)), np.linalg.det(v) * np.linalg.det(w),
                       rtol=1e-12)
    u = fields.gauge_field((2, 2, 2, 2), "haar", 603).reshape(-1, 3, 3)
    p = su3.mul(u[:32], su3.dag(u[32:]))
    assert np.allclose(su3.mul(p, su3.dag(p)), np.eye(3), atol=1e-13)
    assert np.allclose(np.linalg.det(p), 1.0, atol=1e-13)


def test_spinor_product_acts_on_colour_only():
    rng = fields.rng(604)
    u = fields.complex_gaussian(rng, (3, 3, 3))
    psi = fields.complex_gaussian(rng, (3, 4, 3))
    out = su3.mul_spinor(u, psi)
    for x in range(3):
        for s in range(4):
            assert np.allclose(out[x, s], u[x] @ psi[x, s], atol=1e-14)


def test_paper_element_counts():
    """Section 3: 18 x 16 bytes loaded, 9 x 16 stored (432 bytes), 108 fused
    multiply-adds per element in double precision."""
    assert su3.element_bytes(16) == 432
    assert 4 * su3.element_madds() == 108
