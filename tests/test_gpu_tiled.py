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
from tests.gpu_common import PREC_NAME, TOL, case, log_errors, rel, say

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
            err = log_errors(f"H out parity {out_par} dagger {int(dag)}", lat.to_host(dout, out_par, prec), ref)
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
        err = log_errors(f"Schur dagger {int(dag)}", lat.to_host(dout, evenodd.EVEN, prec), wc.schur(e, dagger=dag))
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


def test_set_tiling_through_the_abi(lq):
    """lq_set_tiling: 64-site tiles of both numberings, set through the C ABI,
    give the oracle's Schur operator (single-RHS FP64 and FP16, and 3 RHS in
    the multi-RHS form); the extents in use are reported; once the gauge
    field is uploaded the tiling is fixed (LQ_ESTATE)."""
    dims = (12, 6, 4, 8)
    say(f"set_tiling dims={dims}")
    u, psi, e, o = case(dims, "smooth", 5)
    lat = lq.Lattice(dims, tile_sites=64, mr_tile_sites=64)
    tiles, mr = lat.tiling()
    say(f"  tiles {tiles}, multi-RHS tiles {mr}")
    assert np.prod(tiles) // 2 <= 64 and np.prod(mr) // 2 <= 64
    assert all(d % t == 0 and t % 2 == 0 for d, t in zip(dims, tiles))
    lat.upload_gauge(u)
    lat.set_clover(KAPPA, CSW)
    wc = evenodd.WilsonClover(u, KAPPA, CSW)
    for prec in (0, 2):
        din = lat.to_device(e, evenodd.EVEN, prec)
        dout = lat.new_field(evenodd.EVEN, prec)
        tmp = lat.new_field(evenodd.ODD, prec)
        lat.schur(dout, din, tmp, False, prec)
        err = log_errors(f"Schur {PREC_NAME[prec]}", lat.to_host(dout, evenodd.EVEN, prec),
                         wc.schur(e))
        assert err <= TOL[prec]
    g = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 91, nrhs=3)
    es = np.stack([evenodd.split(g[r], dims)[0] for r in range(3)])
    din = lat.to_device(es, evenodd.EVEN, lq.F16X)
    dout = lat.new_field(evenodd.EVEN, lq.F16X, 3)
    tmp = lat.new_field(evenodd.ODD, lq.F16X, 3)
    lat.schur(dout, din, tmp, False, lq.F16X, 3)
    got = lat.to_host(dout, evenodd.EVEN, lq.F16X, 3)
    for r in range(3):
        assert log_errors(f"multi-RHS Schur rhs {r}", got[r], wc.schur(es[r])) <= TOL[2]
    with pytest.raises(lq.LQError) as ei:
        lat.set_tiling(4096, 0)
    assert ei.value.code == -5


def test_tune_tiles_and_cache(lq, tmp_path):
    """lq_tune_tiles on 16^3x32: every distinct candidate is timed and the
    fastest chosen; the choice is written to the cache file and read back
    from it; the single-RHS and the multi-RHS choice live side by side in
    the file; a context created with the choices uses those tiles."""
    dims = (16, 16, 16, 32)
    path = tmp_path / "tiles.json"
    say(f"tune tiles dims={dims}")
    r1 = lq.tune_tiles(dims, 2, 1, path)
    say(f"  single-RHS FP16: {r1.as_dict()}")
    assert 2 <= r1.ncand <= lq.TUNE_MAX and not r1.from_cache
    us = [r1.us[i] for i in range(r1.ncand)]
    assert min(us) > 0 and r1.us[r1.best] == min(us)
    r2 = lq.tune_tiles(dims, 2, 1, path)
    assert r2.from_cache and r2.best == r1.best
    r3 = lq.tune_tiles(dims, lq.F16X, 12, path)
    say(f"  12-RHS: {r3.as_dict()}")
    assert r3.ncand >= 2 and not r3.from_cache
    text = open(path).read()
    assert ":f16:nrhs1:16x16x16x32" in text and ":f16x:nrhs12:16x16x16x32" in text
    lat = lq.Lattice(dims, tile_sites=r1.target[r1.best], mr_tile_sites=r3.target[r3.best])
    tiles, mr = lat.tiling()
    assert tiles == list(r1.tiles[r1.best]) and mr == list(r3.tiles[r3.best])
    with pytest.raises(lq.LQError):
        lq.tune_tiles(dims, lq.F16X, 17)
