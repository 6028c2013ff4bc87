"""Parity in the tiled site numbering, on lattices small enough for the
oracle.

LQ_TILE_SITES (read when a context is created) caps the sites of one parity
per tile. With 64, an 8x4x4x8 lattice is cut into 8 tiles and a 12x6x4x8
lattice into 18 tiles (3 in x and y), so hops cross tile edges inside the
lattice as well as the lattice boundary. Every kernel of the single-lattice
path walks this numbering. The production volume uses 65536-site tiles,
where the oracle can only be sampled.

Also covered: the FP16 form of the learned preconditioner on half volumes
that leave a partial workgroup and a partial 64-site block, and on
extent-2 directions (both hops of a direction reach the same neighbour).
"""
import numpy as np
import pytest

from gen import fields
from oracle import dirac, evenodd
from oracle import net as onet
from tests.gpu_common import PREC_NAME, TOL, case, rel, say

pytestmark = pytest.mark.gpu

TILED = [(8, 4, 4, 8), (12, 6, 4, 8)]
KAPPA, CSW = 0.135, 1.0


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def tiled_lattice(lq, monkeypatch, dims, u):
    """A context in tiles of at most 64 sites per parity; checks that its
    device order differs from the untiled one (the tiles are in effect)."""
    monkeypatch.setenv("LQ_TILE_SITES", "64")
    lat = lq.Lattice(dims)
    monkeypatch.delenv("LQ_TILE_SITES")
    plain = lq.Lattice(dims)
    probe = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 90)
    e = evenodd.split(probe, dims)[0]
    a = lat.to_device(e, evenodd.EVEN, 0)
    b = plain.to_device(e, evenodd.EVEN, 0)
    assert not bool((a == b).all()), "the tile setting had no effect"
    lat.upload_gauge(u)
    return lat


@pytest.mark.parametrize("dims", TILED)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_operator_parity_tiled(lq, monkeypatch, dims, prec):
    """Hopping term (both parities, and daggers), clover term and Schur
    operator against the oracle."""
    say(f"tiled operator parity dims={dims} prec={PREC_NAME[prec]}")
    u, psi, e, o = case(dims, "smooth", 5)
    lat = tiled_lattice(lq, monkeypatch, dims, u)
    lat.set_clover(KAPPA, CSW)
    wc = evenodd.WilsonClover(u, KAPPA, CSW)
    for out_par, src in ((evenodd.EVEN, o), (evenodd.ODD, e)):
        for dag in (False, True):
            ref = wc.hop_block(src, out_par, dagger=dag)
            dout = lat.new_field(out_par, prec)
            lat.dslash(dout, lat.to_device(src, 1 - out_par, prec), out_par, dag, prec)
            err = rel(lat.to_host(dout, out_par, prec), ref)
            assert err <= TOL[prec], ("dslash", out_par, dag, err)
    ref = wc.clover_half(o, evenodd.ODD, inverse=True)
    dout = lat.new_field(evenodd.ODD, prec)
    lat.clover(dout, lat.to_device(o, evenodd.ODD, prec), evenodd.ODD, True, prec)
    assert rel(lat.to_host(dout, evenodd.ODD, prec), ref) <= TOL[prec]
    din = lat.to_device(e, evenodd.EVEN, prec)
    dout = lat.new_field(evenodd.EVEN, prec)
    tmp = lat.new_field(evenodd.ODD, prec)
    for dag in (False, True):
        lat.schur(dout, din, tmp, dag, prec)
        err = rel(lat.to_host(dout, evenodd.EVEN, prec), wc.schur(e, dagger=dag))
        assert err <= TOL[prec], ("schur", dag, err)


@pytest.mark.parametrize("dims", TILED)
@pytest.mark.parametrize("inner", [0, 2])
def test_solve_tiled(lq, monkeypatch, dims, inner):
    """The CG iteration kernels in the tiled numbering: the solution's
    residual by the oracle's operator."""
    say(f"tiled solve dims={dims} inner={PREC_NAME[inner]}")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 6)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 6)
    lat = tiled_lattice(lq, monkeypatch, dims, u)
    x, rep = lat.solve(b, KAPPA, CSW, 1e-10, inner_prec=inner)
    wc = evenodd.WilsonClover(u, KAPPA, CSW)
    res = dirac.norm(b - wc.M(x.reshape(b.shape))) / dirac.norm(b)
    assert res <= 1e-10, (res, rep)
    assert rep[0].fallback == 0


def random_weights(nl, seed, scale=0.25):
    r = fields.rng(seed)
    return scale * (r.standard_normal((nl, onet.NK, 4, 4))
                    + 1j * r.standard_normal((nl, onet.NK, 4, 4)))


def net_case(lq, lat, u, dims, fp16, adjoint):
    w = random_weights(4, 17)
    net = lq.Net(lat, 4)
    net.set_weights(w)
    full = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 7)
    x = evenodd.split(full, dims)[0]
    dy = lat.new_field(evenodd.EVEN, 1)
    net.apply(dy, lat.to_device(x, evenodd.EVEN, 1), adjoint=adjoint, fp16=fp16)
    got = lat.to_host(dy, evenodd.EVEN, 1)
    if not adjoint:
        ref = onet.apply_even(u, w, x, dims)
    else:
        xf = evenodd.join(x, None, dims)
        ref = evenodd.split(onet.backward(u, w, onet.forward(u, w, xf), xf)[1], dims)[0]
    return rel(got, ref)


@pytest.mark.parametrize("dims", TILED)
@pytest.mark.parametrize("fp16", [False, True])
def test_net_tiled(lq, monkeypatch, dims, fp16):
    """The net's layers (FP32 form, and the solvers' FP16 form) forward and
    adjoint; bounds as in the untiled tests (FP32 rounding of four layers,
    and FP16 rounding of links, activations, weights and transported
    spinors)."""
    say(f"tiled net dims={dims} fp16={fp16}")
    u, _, _, _ = case(dims, "smooth", 8)
    lat = tiled_lattice(lq, monkeypatch, dims, u)
    for adj in (False, True):
        err = net_case(lq, lat, u, dims, fp16, adj)
        assert err <= (5e-3 if fp16 else 2e-5), (adj, err)


@pytest.mark.parametrize("dims", [(6, 2, 2, 2), (6, 4, 2, 10), (2, 2, 2, 2)])
def test_net_fp16_ragged_and_extent_two(lq, dims):
    """FP16 form where the half volume (24, 240, 8 sites) leaves a partial
    workgroup of 128 and a partial block of 64, and where extent-2
    directions send both hops of a direction to one neighbour."""
    say(f"net fp16 dims={dims}")
    u, _, _, _ = case(dims, "smooth", 9)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    for adj in (False, True):
        err = net_case(lq, lat, u, dims, True, adj)
        assert err <= 5e-3, (adj, err)
