"""GPU parity of the hopping term, clover term and Schur operator against the
FP64 oracle, through the C ABI (liblq.so) on the same seeded inputs.

Sizes: tiny lattices with a ragged last block of 64 sites and a ragged last
workgroup, a lattice spanning many workgroups, and the production 32^3x64
volume checked on sampled output sites computed one by one by the oracle.
"""
import numpy as np
import pytest

from gen import fields
from oracle import dirac, evenodd
from tests.gpu_common import PREC_NAME, TOL, case, log_errors, rel, say

pytestmark = pytest.mark.gpu

SMALL = [(4, 4, 4, 4), (6, 2, 2, 2), (10, 6, 4, 6), (2, 2, 2, 2)]
MEDIUM = [(16, 16, 16, 32)]


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def make(lq, dims, kind="smooth", seed=0, kappa=None, csw=None):
    u, psi, e, o = case(dims, kind, seed)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    if kappa is not None:
        lat.set_clover(kappa, csw)
    return lat, u, psi, e, o


@pytest.mark.parametrize("dims", SMALL + MEDIUM)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dslash_parity(lq, dims, prec):
    say(f"dslash parity dims={dims} prec={PREC_NAME[prec]}")
    lat, u, psi, e, o = make(lq, dims, "haar" if dims == (4, 4, 4, 4) else "smooth")
    wc = evenodd.WilsonClover(u, 0.12, 0.0)
    for out_par, src in ((evenodd.EVEN, o), (evenodd.ODD, e)):
        for dag in (False, True):
            ref = wc.hop_block(src, out_par, dagger=dag)
            din = lat.to_device(src, 1 - out_par, prec)
            dout = lat.new_field(out_par, prec)
            lat.dslash(dout, din, out_par, dag, prec)
            got = lat.to_host(dout, out_par, prec)
            err = log_errors(f"H out parity {out_par} dagger {int(dag)}", got, ref)
            assert err <= TOL[prec], (dims, prec, out_par, dag, err)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dslash_parity_32x64_sampled(lq, prec):
    """Production volume: sampled output sites against the per-site oracle."""
    dims = (32, 32, 32, 64)
    say(f"dslash sampled parity dims={dims} prec={PREC_NAME[prec]}")
    lat, u, psi, e, o = make(lq, dims, "smooth", seed=2)
    din = lat.to_device(e, evenodd.EVEN, prec)
    dout = lat.new_field(evenodd.ODD, prec)
    for dag in (False, True):
        lat.dslash(dout, din, evenodd.ODD, dag, prec)
        got = lat.to_host(dout, evenodd.ODD, prec)
        full_in = evenodd.join(e, None, dims)
        rng = fields.rng(99)
        lx, ly, lz, lt = dims
        sites = [(1, 0, 0, 0), (lx - 1, ly - 1, lz - 1, lt - 1), (0, 0, 0, lt - 1)]
        while len(sites) < 40:
            c = [int(rng.integers(d)) for d in dims]
            if sum(c) % 2 == 1:
                sites.append(tuple(c))
        num = den = 0.0
        for x in sites:
            if sum(x) % 2 != 1:
                continue
            i = ((x[3] * lz + x[2]) * ly + x[1]) * lx + x[0]
            ref = dirac.hop_at(u, full_in, x, dagger=dag)
            num += np.sum(np.abs(got[i // 2] - ref) ** 2)
            den += np.sum(np.abs(ref) ** 2)
        err = np.sqrt(num / den)
        assert err <= TOL[prec], (prec, dag, err)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (10, 6, 4, 6), (16, 16, 16, 32)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_clover_and_schur_parity(lq, dims, prec):
    say(f"clover/schur parity dims={dims} prec={PREC_NAME[prec]}")
    kappa, csw = 0.135, 1.0
    lat, u, psi, e, o = make(lq, dims, "smooth", seed=1, kappa=kappa, csw=csw)
    wc = evenodd.WilsonClover(u, kappa, csw)
    # clover term and its inverse
    forms = [(evenodd.EVEN, False, e), (evenodd.ODD, True, o)]
    if prec == 0:
        forms += [(evenodd.ODD, False, o), (evenodd.EVEN, True, e)]
    for par, inv, src in forms:
        ref = wc.clover_half(src, par, inverse=inv)
        din = lat.to_device(src, par, prec)
        dout = lat.new_field(par, prec)
        lat.clover(dout, din, par, inv, prec)
        err = log_errors(f"clover parity {par} inverse {int(inv)}",
                         lat.to_host(dout, par, prec), ref)
        assert err <= TOL[prec], ("clover", par, inv, err)
    # Schur operator and its adjoint
    din = lat.to_device(e, evenodd.EVEN, prec)
    dout = lat.new_field(evenodd.EVEN, prec)
    tmp = lat.new_field(evenodd.ODD, prec)
    for dag in (False, True):
        ref = wc.schur(e, dagger=dag)
        lat.schur(dout, din, tmp, dag, prec)
        err = log_errors(f"Schur dagger {int(dag)}", lat.to_host(dout, evenodd.EVEN, prec), ref)
        assert err <= TOL[prec], ("schur", dag, err)


def test_dslash_fp64_deterministic(lq):
    dims = (16, 16, 16, 32)
    say(f"dslash determinism dims={dims}")
    lat, u, psi, e, o = make(lq, dims)
    din = lat.to_device(o, evenodd.ODD, 0)
    a = lat.new_field(evenodd.EVEN, 0)
    b = lat.new_field(evenodd.EVEN, 0)
    lat.dslash(a, din, evenodd.EVEN, False, 0)
    lat.dslash(b, din, evenodd.EVEN, False, 0)
    assert bool((a == b).all())


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_norm_dot_parity(lq, prec):
    dims = (10, 6, 4, 6)
    say(f"norm/dot parity dims={dims} prec={PREC_NAME[prec]}")
    lat, u, psi, e, o = make(lq, dims)
    e2 = evenodd.split(fields.gaussian_spinor(dims, 77), dims)[0]
    da = lat.to_device(e, evenodd.EVEN, prec)
    db = lat.to_device(e2, evenodd.EVEN, prec)
    # compare with the values of the rounded device fields
    ha = lat.to_host(da, evenodd.EVEN, prec)
    hb = lat.to_host(db, evenodd.EVEN, prec)
    n = lat.norm2(da, evenodd.EVEN, prec)
    d = lat.dot(da, db, evenodd.EVEN, prec)
    assert abs(n - np.vdot(ha, ha).real) <= 1e-13 * n
    ref = np.vdot(ha, hb)
    assert abs(d - ref) <= 1e-13 * np.sqrt(n * np.vdot(hb, hb).real)


def test_spinor_roundtrip_full_and_rhs(lq):
    dims = (6, 2, 2, 2)
    say(f"spinor round trip dims={dims}")
    lat, u, psi, e, o = make(lq, dims)
    two = np.stack([psi, 2 * psi])
    d = lat.to_device(two, 2, 0)
    back = lat.to_host(d, 2, 0, nrhs=2)
    assert np.array_equal(back.reshape(two.shape), two)


def test_gauge_upload_rejects_non_su3(lq):
    dims = (4, 4, 4, 4)
    say("gauge upload rejects a non-SU(3) field")
    u = fields.gauge_field(dims, "haar", 5).copy()
    u[1, 2, 3, 0, 2] *= -1.0  # det = -1
    lat = lq.Lattice(dims)
    with pytest.raises(lq.LQError) as ei:
        lat.upload_gauge(u)
    assert ei.value.code == -1
    with pytest.raises(lq.LQError):
        lat.dslash(lat.new_field(0, 0), lat.new_field(1, 0), 0)
