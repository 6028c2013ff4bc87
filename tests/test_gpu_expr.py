"""GPU parity of the fused site-local expressions (lq_su3_mul,
lq_su3_spinor_mul) against the oracle's plain definitions (oracle/su3.py):
FP64 to rounding (1e-14 relative), FP32 to 1e-6, on element counts that
leave a ragged last block; the three-factor product in one pass; output
aliasing an input; bad arguments."""
import numpy as np
import pytest

from gen import fields
from oracle import su3
from tests.gpu_common import rel, say

pytestmark = pytest.mark.gpu

TOL = {0: 1e-14, 1: 1e-6}


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def mats(n, seed):
    return fields.complex_gaussian(fields.rng(seed), (n, 3, 3))


@pytest.mark.parametrize("n", [1, 64, 1000, 64 * 37 + 5])
@pytest.mark.parametrize("prec", [0, 1])
def test_su3_mul_forms(lq, n, prec):
    say(f"su3 mul n={n} prec={prec}")
    v, w, x = mats(n, 610), mats(n, 611), mats(n, 612)
    dv = lq.site_array_to_device(v, lq.SITE_SU3, prec)
    dw = lq.site_array_to_device(w, lq.SITE_SU3, prec)
    dx = lq.site_array_to_device(x, lq.SITE_SU3, prec)
    du = lq.site_array_to_device(np.zeros_like(v), lq.SITE_SU3, prec)
    refs = {lq.SU3_VW: su3.mul(v, w), lq.SU3_VWDAG: su3.mul(v, su3.dag(w)),
            lq.SU3_VDAGW: su3.mul(su3.dag(v), w), lq.SU3_VWX: su3.mul(su3.mul(v, w), x)}
    for form, ref in refs.items():
        lq.su3_mul(du, dv, dw, n, form, prec, x=dx)
        got = lq.site_array_to_host(du, n, lq.SITE_SU3, prec)
        assert rel(got, ref) <= TOL[prec] * (3 if form == lq.SU3_VWX else 1), form


def test_su3_mul_in_place_and_su3_closure(lq):
    """U = V W with U the same array as V; products of Haar SU(3) links stay
    unitary with determinant 1 to FP64 rounding."""
    u = fields.gauge_field((4, 4, 4, 4), "haar", 613).reshape(-1, 3, 3)
    n = u.shape[0] // 2
    v, w = u[:n].copy(), u[n:].copy()
    dv = lq.site_array_to_device(v, lq.SITE_SU3, 0)
    dw = lq.site_array_to_device(w, lq.SITE_SU3, 0)
    lq.su3_mul(dv, dv, dw, n, lq.SU3_VWDAG, 0)
    got = lq.site_array_to_host(dv, n, lq.SITE_SU3, 0)
    assert rel(got, su3.mul(v, su3.dag(w))) <= 1e-14
    assert np.allclose(su3.mul(got, su3.dag(got)), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(got), 1.0, atol=1e-14)


@pytest.mark.parametrize("prec", [0, 1])
def test_su3_spinor_mul(lq, prec):
    n = 64 * 9 + 17
    u = mats(n, 614)
    psi = fields.complex_gaussian(fields.rng(615), (n, 4, 3))
    du = lq.site_array_to_device(u, lq.SITE_SU3, prec)
    dp = lq.site_array_to_device(psi, lq.SITE_SPINOR, prec)
    do = lq.site_array_to_device(np.zeros_like(psi), lq.SITE_SPINOR, prec)
    for adj in (False, True):
        lq.su3_spinor_mul(do, du, dp, n, adj, prec)
        got = lq.site_array_to_host(do, n, lq.SITE_SPINOR, prec)
        ref = su3.mul_spinor(su3.dag(u) if adj else u, psi)
        assert rel(got, ref) <= TOL[prec]


def test_su3_mul_rejects_bad_arguments(lq):
    dv = lq.site_array_to_device(mats(8, 616), lq.SITE_SU3, 0)
    for form, prec in [(7, 0), (0, 2), (lq.SU3_VWX, 0)]:  # VWX without x
        with pytest.raises(lq.LQError):
            lq.su3_mul(dv, dv, dv, 8, form, prec)
