"""GPU tests of the uneven batch (lq_ensemble_*): independent Wilson-clover
solves on lattices of different extents and hopping parameters advanced
together, checked member by member against the FP64 oracle.

Small batches are checked with the oracle's whole-lattice residual
||b - M x|| / ||b||; the batch of eight lattices from 8^4 to 24^3x48 that the
benchmark times is checked with the library's FP64 true residual and, at
sampled sites of every member, with the oracle's single-site residual.
"""
import json

import numpy as np
import pytest

from gen import fields
from oracle import dirac, evenodd
from tests.gpu_common import residual_at, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def make_members(lq, spec, csw=1.0, clover=True):
    """spec: list of (dims, kappa, gauge seed, source seed)."""
    lats, us, bs, dev_b, dev_x = [], [], [], [], []
    for dims, kappa, gs, ss in spec:
        u = fields.gauge_field(dims, "smooth", gs)
        lat = lq.Lattice(dims)
        lat.upload_gauge(u)
        if clover:
            lat.set_clover(kappa, csw)
        b = fields.gaussian_spinor(dims, ss)
        lats.append(lat)
        us.append(u)
        bs.append(b)
        dev_b.append(lat.to_device(b, lq.FULL, lq.F64))
        dev_x.append(lat.new_field(lq.FULL, lq.F64))
    return lats, us, bs, dev_b, dev_x


def oracle_residual(u, kappa, csw, x, b):
    return dirac.norm(b - evenodd.WilsonClover(u, kappa, csw).M(x)) / dirac.norm(b)


SMALL = [((4, 4, 4, 4), 0.125, fields.SEED_GAUGE + 40, fields.SEED_SOURCE + 40),
         ((8, 8, 8, 8), 0.132, fields.SEED_GAUGE + 41, fields.SEED_SOURCE + 41),
         ((6, 4, 4, 8), 0.128, fields.SEED_GAUGE + 42, fields.SEED_SOURCE + 42),
         ((10, 6, 4, 6), 0.135, fields.SEED_GAUGE + 43, fields.SEED_SOURCE + 43)]


@pytest.mark.parametrize("inner", [2, 1, 0])
def test_small_uneven_batch(lq, inner):
    """Every member reaches the tolerance by the oracle's residual, the
    library's reported residual agrees with it, and the iteration counts
    stay close to the same solver run one lattice at a time."""
    tol, csw = 1e-10, 1.0
    say(f"uneven batch small inner={inner}")
    lats, us, bs, db, dx = make_members(lq, SMALL, csw)
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _, _ in SMALL]
    reps, er = ens.solve_device(dx, db, kap, [csw] * len(lats), tol, inner_prec=inner)
    say(f"  batch {er}")
    assert er["tile_sites"] in (64, 128, 256)
    for j, lat in enumerate(lats):
        x = lat.to_host(dx[j], lq.FULL, lq.F64).reshape(bs[j].shape)
        res = oracle_residual(us[j], kap[j], csw, x, bs[j])
        xs, rs = lat.solve(bs[j], kap[j], csw, tol, inner_prec=inner)
        say(f"  member {j} dims={lat.dims} it={reps[j].iterations} single it={rs[0].iterations} "
            f"upd={reps[j].reliable_updates} fb={reps[j].fallback} res={res:.3e}")
        assert res <= tol, (j, res)
        assert abs(reps[j].true_residual - res) <= 0.1 * res + 1e-14
        assert reps[j].fallback == 0
        assert abs(reps[j].iterations - rs[0].iterations) <= max(5, rs[0].iterations // 10)
        err = np.linalg.norm((x - xs).reshape(-1)) / np.linalg.norm(xs.reshape(-1))
        assert err <= 1e3 * tol, (j, err)
    ens.close()


def test_dropout_zero_source_and_reuse(lq):
    """Members converging at very different rates (the fast ones leave the
    tile list, so the graph is captured again) and a zero source (x = 0);
    a second solve on the same batch reuses its tile choice."""
    tol, csw = 1e-10, 1.0
    spec = [((8, 8, 8, 8), 0.100, fields.SEED_GAUGE + 44, fields.SEED_SOURCE + 44),
            ((8, 8, 8, 8), 0.136, fields.SEED_GAUGE + 45, fields.SEED_SOURCE + 45),
            ((4, 4, 4, 4), 0.110, fields.SEED_GAUGE + 46, fields.SEED_SOURCE + 46),
            ((6, 6, 6, 6), 0.120, fields.SEED_GAUGE + 47, fields.SEED_SOURCE + 47)]
    say("uneven batch drop-out")
    lats, us, bs, db, dx = make_members(lq, spec, csw)
    bs[3][:] = 0.0
    db[3] = lats[3].to_device(bs[3], lq.FULL, lq.F64)
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _, _ in spec]
    for rep_no in range(2):
        reps, er = ens.solve_device(dx, db, kap, [csw] * 4, tol, inner_prec=lq.F16,
                                    check_every=4)
        say(f"  solve {rep_no}: {er} iters={[r.iterations for r in reps]}")
        assert reps[0].iterations < reps[1].iterations
        if rep_no == 0:
            assert er["graph_captures"] >= 2
        for j in range(3):
            x = lats[j].to_host(dx[j], lq.FULL, lq.F64).reshape(bs[j].shape)
            assert oracle_residual(us[j], kap[j], csw, x, bs[j]) <= tol
        assert np.all(lats[3].to_host(dx[3], lq.FULL, lq.F64) == 0)
        assert reps[3].iterations == 0 and reps[3].true_residual == 0.0
    ens.close()


def test_mixed_boundaries_and_extent_two(lq):
    """Members differ in their time boundary (one periodic) and include an
    extent-2 direction (both hops of that direction land on one site and
    add); each is checked against the oracle with its own boundary."""
    tol, csw = 1e-10, 1.0
    say("uneven batch: periodic member and extent-2 member")
    spec = [((4, 4, 4, 4), 0.12, False), ((6, 2, 2, 2), 0.11, True), ((8, 4, 4, 8), 0.125, True)]
    lats, us, bs, db, dx = [], [], [], [], []
    for j, (dims, kappa, apt) in enumerate(spec):
        u = fields.gauge_field(dims, "haar" if j == 1 else "smooth", fields.SEED_GAUGE + 50 + j)
        lat = lq.Lattice(dims, antiperiodic_t=apt)
        lat.upload_gauge(u)
        lat.set_clover(kappa, csw)
        b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 50 + j)
        lats.append(lat)
        us.append(u)
        bs.append(b)
        db.append(lat.to_device(b, lq.FULL, lq.F64))
        dx.append(lat.new_field(lq.FULL, lq.F64))
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _ in spec]
    reps, er = ens.solve_device(dx, db, kap, [csw] * 3, tol, inner_prec=lq.F16)
    say(f"  {er} iters={[r.iterations for r in reps]}")
    for j, (dims, kappa, apt) in enumerate(spec):
        x = lats[j].to_host(dx[j], lq.FULL, lq.F64).reshape(bs[j].shape)
        wc = evenodd.WilsonClover(us[j], kappa, csw, antiperiodic_t=apt)
        res = dirac.norm(bs[j] - wc.M(x)) / dirac.norm(bs[j])
        assert res <= tol, (j, res)
    ens.close()


def test_without_graph_same_result(lq):
    """use_graph = -1 launches the same kernels one by one: the same
    iteration counts and residuals within the tolerance."""
    tol, csw = 1e-10, 1.0
    say("uneven batch no graph")
    lats, us, bs, db, dx = make_members(lq, SMALL[:2], csw)
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _, _ in SMALL[:2]]
    r1, _ = ens.solve_device(dx, db, kap, [csw] * 2, tol, inner_prec=lq.F32)
    x1 = [l.to_host(d, lq.FULL, lq.F64) for l, d in zip(lats, dx)]
    r2, e2 = ens.solve_device(dx, db, kap, [csw] * 2, tol, inner_prec=lq.F32, use_graph=-1)
    assert e2["graph_captures"] == 0
    for j in range(2):
        x2 = lats[j].to_host(dx[j], lq.FULL, lq.F64)
        # same kernels, same reduction order: the same solution
        assert r1[j].iterations == r2[j].iterations
        assert np.array_equal(x1[j], x2)
    ens.close()


def test_fault_injection_falls_back(lq):
    """Members of even index withhold their inner corrections: their FP64
    residual cannot fall, the stagnation test stops them, and the FP64 CG of
    their own context finishes them; the other members finish in the batch."""
    tol, csw = 1e-10, 1.0
    say("uneven batch fault injection")
    lats, us, bs, db, dx = make_members(lq, SMALL, csw)
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _, _ in SMALL]
    reps, er = ens.solve_device(dx, db, kap, [csw] * 4, tol, inner_prec=lq.F16, fault_inject=1)
    say(f"  {er} fallback={[r.fallback for r in reps]}")
    assert [r.fallback for r in reps] == [1, 0, 1, 0]
    for j in range(4):
        x = lats[j].to_host(dx[j], lq.FULL, lq.F64).reshape(bs[j].shape)
        assert oracle_residual(us[j], kap[j], csw, x, bs[j]) <= tol
    with pytest.raises(lq.LQError):
        ens.solve_device(dx, db, kap, [csw] * 4, tol, inner_prec=lq.F64, fault_inject=1)
    ens.close()


def test_maxiter_reports_noconv(lq):
    say("uneven batch maxiter")
    lats, us, bs, db, dx = make_members(lq, SMALL[:2], 1.0)
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _, _ in SMALL[:2]]
    with pytest.raises(lq.LQError) as ei:
        ens.solve_device(dx, db, kap, [1.0, 1.0], 1e-10, inner_prec=lq.F16, maxiter=3)
    assert "ENOCONV" in str(ei.value)
    reps, _ = ens.solve_device(dx, db, kap, [1.0, 1.0], 1e-10, inner_prec=lq.F16, maxiter=3,
                               raise_on_noconv=False)
    for r in reps:
        assert r.true_residual > 1e-10
    ens.close()


def test_bad_arguments(lq):
    say("uneven batch bad arguments")
    lats, us, bs, db, dx = make_members(lq, SMALL[:2], 1.0, clover=False)
    with pytest.raises(lq.LQError):
        lq.Ensemble([lats[0], lats[0]])
    ens = lq.Ensemble(lats)
    with pytest.raises(lq.LQError) as ei:
        ens.tune(lq.F16)  # no clover term yet
    assert "ESTATE" in str(ei.value)
    with pytest.raises(lq.LQError):
        ens.solve_device(dx, db, [0.12, 0.3], [1.0, 1.0], 1e-10)  # kappa out of range
    with pytest.raises(lq.LQError):
        ens.solve_device(dx, db, [0.12, 0.12], [1.0, 1.0], 1e-10, inner_prec=7)
    with pytest.raises(lq.LQError):
        ens.solve_device(dx, dx, [0.12, 0.12], [1.0, 1.0], 1e-10)  # aliased fields
    ens.close()


def test_tile_cache_file(lq, tmp_path):
    """A measured choice is written to the cache file; a new batch of the
    same extents reads it back instead of measuring; an entry edited by hand
    is obeyed."""
    path = str(tmp_path / "tiles.json")
    say("uneven batch tile cache")
    lats, us, bs, db, dx = make_members(lq, SMALL, 1.0)
    e1 = lq.Ensemble(lats)
    t1 = e1.tune(lq.F16, path)
    say(f"  measured {t1}")
    assert t1["tile_from_cache"] == 0
    assert t1["tile_sites"] in (64, 128, 256)
    assert all(m > 0 for m in t1["tune_ms"])
    assert t1["tile_sites"] == (64, 128, 256)[int(np.argmin(t1["tune_ms"]))]
    data = json.load(open(path))
    (key,) = data.keys()
    assert ":f16:nrhs1:4x4x4x4+8x8x8x8+6x4x4x8+10x6x4x6" in key
    assert key.startswith("gfx")
    e1.close()
    e2 = lq.Ensemble(lats)
    t2 = e2.tune(lq.F16, path)
    assert t2["tile_from_cache"] == 1 and t2["tile_sites"] == t1["tile_sites"]
    e2.close()
    forced = 64 if t1["tile_sites"] != 64 else 128
    data[key]["tile_sites"] = forced
    json.dump(data, open(path, "w"))
    e3 = lq.Ensemble(lats)
    t3 = e3.tune(lq.F16, path)
    assert t3["tile_from_cache"] == 1 and t3["tile_sites"] == forced
    # the solve uses the tile held in memory
    kap = [k for _, k, _, _ in SMALL]
    reps, er = e3.solve_device(dx, db, kap, [1.0] * 4, 1e-10, inner_prec=lq.F16)
    assert er["tile_sites"] == forced
    for j in range(4):
        x = lats[j].to_host(dx[j], lq.FULL, lq.F64).reshape(bs[j].shape)
        assert oracle_residual(us[j], kap[j], 1.0, x, bs[j]) <= 1e-10
    # another precision is a separate entry
    t4 = e3.tune(lq.F32, path)
    assert t4["tile_from_cache"] == 0
    assert len(json.load(open(path))) == 2
    e3.close()


def test_full_uneven_batch(lq):
    """The eight lattices of the benchmark (8^4 ... 24^3x48, kappa in
    [0.130, 0.136], csw = 1), FP16 inner iteration: every member converges
    without fallback; the two smallest are checked with the oracle's
    whole-lattice residual, every member at sampled sites with the oracle's
    single-site residual."""
    tol, csw = 1e-10, 1.0
    spec = fields.uneven_batch()
    say(f"uneven batch full: {[d for d, *_ in spec]}")
    lats, us, bs, db, dx = make_members(lq, spec, csw)
    ens = lq.Ensemble(lats)
    kap = [k for _, k, _, _ in spec]
    reps, er = ens.solve_device(dx, db, kap, [csw] * len(spec), tol, inner_prec=lq.F16)
    say(f"  {er}")
    rng = np.random.default_rng(11)
    for j, lat in enumerate(lats):
        r = reps[j]
        say(f"  member {j} dims={lat.dims} kappa={kap[j]:.4f} it={r.iterations} "
            f"upd={r.reliable_updates} fb={r.fallback} res={r.true_residual:.3e}")
        assert r.true_residual <= tol and r.fallback == 0
        x = lat.to_host(dx[j], lq.FULL, lq.F64).reshape(bs[j].shape)
        if np.prod(lat.dims) <= 12 ** 3 * 24:
            assert oracle_residual(us[j], kap[j], csw, x, bs[j]) <= tol
        bn = dirac.norm(bs[j]) / np.sqrt(np.prod(lat.dims))  # RMS site norm of b
        for _ in range(8):
            site = tuple(int(rng.integers(0, L)) for L in lat.dims)
            rs = np.linalg.norm(residual_at(us[j], kap[j], csw, x, bs[j], site))
            assert rs <= 1e3 * tol * bn, (j, site, rs / bn)
    ens.close()
