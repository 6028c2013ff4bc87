"""GPU solves of M x = b (through lq_solve) checked by the FP64 oracle: the
true residual is recomputed with the oracle's own operator, and on small
lattices the solution is compared with a direct sparse LU solve of the
brute-force matrix."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import fields
from oracle import dirac, evenodd
from tests import bruteforce
from tests.gpu_common import case, residual_at, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def oracle_residual(u, kappa, csw, x, b):
    wc = evenodd.WilsonClover(u, kappa, csw)
    return dirac.norm(b - wc.M(x.reshape(b.shape))) / dirac.norm(b)


def direct(u, dims, kappa, csw, b):
    wc = evenodd.WilsonClover(u, kappa, csw)
    h = bruteforce.hopping_matrix(u, dims)
    a = bruteforce.clover_block_matrix(wc.a.reshape(-1, 12, 12))
    return spla.spsolve((a - kappa * h).tocsc(), b.reshape(-1))


@pytest.mark.parametrize("inner", [0, 1, 2])
def test_config0_wilson_haar_4x4(lq, inner):
    """4^4, Wilson (csw = 0), kappa = 0.12, Haar links, Gaussian source."""
    dims, kappa, csw = (4, 4, 4, 4), 0.12, 0.0
    say(f"solve 4^4 wilson inner={inner}")
    u = fields.gauge_field(dims, "haar", fields.SEED_GAUGE)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, inner_prec=inner)
    res = oracle_residual(u, kappa, csw, x, b)
    assert res <= 1e-10, (res, rep)
    assert abs(rep[0].true_residual - res) <= 0.1 * res + 1e-14
    xr = direct(u, dims, kappa, csw, b)
    err = np.linalg.norm(x.reshape(-1) - xr) / np.linalg.norm(xr)
    assert err <= 4 * 1e-10 * 4, err  # cond(M) ~ 4 at this kappa


@pytest.mark.parametrize("dims", [(10, 6, 4, 6), (8, 8, 8, 8)])
@pytest.mark.parametrize("inner", [0, 1, 2])
def test_clover_smooth_solves(lq, dims, inner):
    kappa, csw = 0.135, 1.0
    say(f"solve clover dims={dims} inner={inner}")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, inner_prec=inner)
    res = oracle_residual(u, kappa, csw, x, b)
    assert res <= 1e-10, (res, rep)
    if inner > 0:
        assert rep[0].reliable_updates >= 1


def test_graph_and_direct_launch_agree(lq):
    dims, kappa, csw = (8, 4, 4, 8), 0.13, 1.0
    say("solve graph vs direct launches")
    u = fields.gauge_field(dims, "smooth", 7)
    b = fields.gaussian_spinor(dims, 8)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x1, r1 = lat.solve(b, kappa, csw, 1e-10, use_graph=0)
    x2, r2 = lat.solve(b, kappa, csw, 1e-10, use_graph=-1)
    assert r1[0].iterations == r2[0].iterations
    assert np.array_equal(x1, x2)


def test_fault_injection_falls_back_to_fp64(lq):
    dims, kappa, csw = (8, 8, 8, 8), 0.135, 1.0
    say("solve with forced stagnation of the mixed-precision inner solve")
    u = fields.gauge_field(dims, "smooth", 9)
    b = fields.gaussian_spinor(dims, 10)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, inner_prec=1, fault_inject=1,
                       raise_on_noconv=False)
    say(f"report {rep[0]}")
    assert rep[0].fallback == 1
    assert oracle_residual(u, kappa, csw, x, b) <= 1e-10


def test_multiple_rhs_and_zero_source(lq):
    dims, kappa, csw = (4, 4, 4, 8), 0.13, 1.0
    say("solve two right-hand sides, one of them zero")
    u = fields.gauge_field(dims, "smooth", 11)
    b = np.stack([fields.gaussian_spinor(dims, 12), np.zeros(u.shape[:4] + (4, 3))])
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, inner_prec=1)
    assert oracle_residual(u, kappa, csw, x[0], b[0]) <= 1e-10
    assert np.all(x[1] == 0)


def test_config1_mixed_fp32_16x32(lq):
    """16^3x32 even-odd Wilson-clover, kappa = 0.135, csw = 1, smooth links,
    FP32 inner CG with FP64 reliable updates, against plain FP64 CG."""
    dims, kappa, csw = (16, 16, 16, 32), 0.135, 1.0
    say("solve 16^3x32 mixed fp32 vs plain fp64")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x64, r64 = lat.solve(b, kappa, csw, 1e-10, inner_prec=0)
    x32, r32 = lat.solve(b, kappa, csw, 1e-10, inner_prec=1)
    for x in (x64, x32):
        assert oracle_residual(u, kappa, csw, x, b) <= 1e-10
    err = np.linalg.norm((x32 - x64).reshape(-1)) / np.linalg.norm(x64.reshape(-1))
    say(f"fp64 {r64[0]}\nfp32 {r32[0]}\nmixed vs plain relative difference {err:.2e}")
    assert err <= 1e-8


@pytest.mark.parametrize("inner", [0, 1, 2])
def test_bicgstab_solves(lq, inner):
    """BiCGStab on the Schur operator: 4^4 Haar Wilson against the direct
    solve, and an 8^4 smooth clover lattice checked by the oracle residual."""
    say(f"bicgstab inner={inner}")
    dims, kappa, csw = (4, 4, 4, 4), 0.12, 0.0
    u = fields.gauge_field(dims, "haar", fields.SEED_GAUGE)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, solver=lq.BICGSTAB, inner_prec=inner)
    assert oracle_residual(u, kappa, csw, x, b) <= 1e-10
    xr = direct(u, dims, kappa, csw, b)
    assert np.linalg.norm(x.reshape(-1) - xr) <= 16e-10 * np.linalg.norm(xr)
    dims, kappa, csw = (8, 8, 8, 8), 0.135, 1.0
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, solver=lq.BICGSTAB, inner_prec=inner)
    say(f"  8^4 clover: {rep[0].iterations} iterations, {rep[0].reliable_updates} restarts")
    assert oracle_residual(u, kappa, csw, x, b) <= 1e-10


@pytest.mark.parametrize("inner", [0, 2])
def test_bicgstab_indefinite_system(lq, inner):
    """At kappa = 0.135 the smooth-link Schur operator is indefinite (the free
    critical kappa is 1/8; these links, <Re tr U>/3 ~ 0.94, move it to ~0.133)
    and textbook BiCGStab stagnates (the oracle's, on this 8^3x16 system, near
    3e-4 for 2000 iterations).  Restarts from the true residual, and the plain
    FP64 CG where BiCGStab still makes no progress, must deliver the solution
    in every inner precision."""
    dims, kappa, csw = (8, 8, 8, 16), 0.135, 1.0
    say(f"bicgstab indefinite inner={inner}")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, solver=lq.BICGSTAB, inner_prec=inner)
    say(f"  {rep[0].iterations} iterations, {rep[0].reliable_updates} restarts, "
        f"fallback {rep[0].fallback}, residual {rep[0].true_residual:.2e}")
    assert oracle_residual(u, kappa, csw, x, b) <= 1e-10


def test_bicgstab_fault_injection_falls_back(lq):
    dims, kappa, csw = (8, 8, 8, 8), 0.135, 1.0
    say("bicgstab with forced stagnation")
    u = fields.gauge_field(dims, "smooth", 9)
    b = fields.gaussian_spinor(dims, 10)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    x, rep = lat.solve(b, kappa, csw, 1e-10, solver=lq.BICGSTAB, inner_prec=1, fault_inject=1,
                       raise_on_noconv=False)
    assert rep[0].fallback == 1
    assert oracle_residual(u, kappa, csw, x, b) <= 1e-10


def sampled_residuals(u, kappa, csw, x, b, extra_sites, n_random, seed):
    """Norms of the oracle's single-site residual (b - M x)(site) at the given
    sites, the lattice corners and n_random random sites."""
    lt, lz, ly, lx = u.shape[:4]
    rng = fields.rng(seed)
    sites = [(0, 0, 0, 0), (lx - 1, ly - 1, lz - 1, lt - 1), (0, 0, 0, lt - 1)] + list(extra_sites)
    sites += [(int(rng.integers(lx)), int(rng.integers(ly)), int(rng.integers(lz)),
               int(rng.integers(lt))) for _ in range(n_random)]
    return [float(np.linalg.norm(residual_at(u, kappa, csw, x, b, s))) for s in sites]


def test_full_size_mixed_solve(lq):
    """The benchmark's step at its full size: 32^3x64, kappa 0.135, csw 1,
    smooth links, Gaussian source, FP16 inner iteration with FP64 reliable
    updates.  No site may carry more than the whole residual allows
    (|r(x)| <= tol |b|), by the oracle's own operator at sampled sites; the
    solution agrees with the plain FP64 solve within the conditioning bound."""
    dims, kappa, csw, tol = (32, 32, 32, 64), 0.135, 1.0, 1e-10
    say("full-size mixed solve 32^3x64")
    u, b, _, _ = case(dims, "smooth", 2)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    db = lat.to_device(b, lq.FULL, lq.F64)
    dx = lat.new_field(lq.FULL, lq.F64)
    rep = lat.solve_device(dx, db, kappa, csw, tol, inner_prec=lq.F16)[0]
    say(f"  {rep.iterations} iterations, {rep.reliable_updates} updates, "
        f"residual {rep.true_residual:.2e}")
    assert rep.true_residual <= tol and rep.fallback == 0
    x = lat.to_host(dx, lq.FULL, lq.F64).reshape(b.shape)
    bound = tol * dirac.norm(b)
    rs = sampled_residuals(u, kappa, csw, x, b, [], 24, 301)
    say(f"  largest sampled site residual {max(rs):.2e} (bound {bound:.2e})")
    assert max(rs) <= 1.01 * bound
    dx64 = lat.new_field(lq.FULL, lq.F64)
    lat.solve_device(dx64, db, kappa, csw, 1e-12, inner_prec=lq.F64)
    x64 = lat.to_host(dx64, lq.FULL, lq.F64).reshape(b.shape)
    err = dirac.norm(x - x64) / dirac.norm(x64)
    say(f"  relative difference to the plain FP64 solution {err:.2e}")
    assert err <= 1e3 * tol


@pytest.mark.parametrize("batched", [1, 2])
def test_full_size_batched_point_sources(lq, batched):
    """The 12 spin-colour point sources at 32^3x64 through the 12-RHS
    operator, as 12 recurrences (batched 1) and as block CG (batched 2):
    every RHS reaches the tolerance without the FP64 fallback, and at the
    origin, its eight neighbours and random sites the oracle's residual of
    each RHS stays within the bound the whole residual sets (|b_r| = 1).
    On this lattice the fronts of the point-source Krylov vectors fall below
    the FP32 normal range within a few iterations, which the FP16 per-site
    scales must store as zero."""
    dims, kappa, csw, tol = (32, 32, 32, 64), 0.135, 1.0, 1e-10
    say(f"full-size point sources 32^3x64 batched={batched}")
    u, _, _, _ = case(dims, "smooth", 2)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    b = fields.point_sources_12(dims)
    x, reps = lat.solve(b, kappa, csw, tol, inner_prec=lq.F16, batched=batched)
    say(f"  {reps[0].iterations} iterations, max residual "
        f"{max(r.true_residual for r in reps):.2e}")
    assert max(r.true_residual for r in reps) <= tol
    assert all(r.fallback == 0 for r in reps)
    lx, ly, lz, lt = dims
    near = [(1, 0, 0, 0), (lx - 1, 0, 0, 0), (0, 1, 0, 0), (0, ly - 1, 0, 0), (0, 0, 1, 0),
            (0, 0, lz - 1, 0), (0, 0, 0, 1)]
    worst = 0.0
    for r in range(12):
        rs = sampled_residuals(u, kappa, csw, x[r].reshape(b[r].shape), b[r], near, 4, 400 + r)
        worst = max(worst, max(rs))
    say(f"  largest sampled site residual {worst:.2e} (bound {tol:.2e})")
    assert worst <= 1.01 * tol



@pytest.mark.parametrize("batched", [0, 1])
def test_reference_error_in_report(lq, batched):
    """With a reference solution on the device the report gives
    ||x - xref|| / ||xref|| per right-hand side; it equals the same norm
    taken on the host, and the mixed solves agree with the FP64 CG to about
    the condition number times the tolerance."""
    dims, kappa, csw, tol = (8, 4, 4, 8), 0.135, 1.0, 1e-10
    say(f"reference error batched={batched}")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 7)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 7, nrhs=2)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    db = lat.to_device(b, lq.FULL, lq.F64)
    dref = lat.new_field(lq.FULL, lq.F64, 2)
    lat.solve_device(dref, db, kappa, csw, 1e-12, nrhs=2, inner_prec=lq.F64)
    dx = lat.new_field(lq.FULL, lq.F64, 2)
    reps = lat.solve_device(dx, db, kappa, csw, tol, nrhs=2, inner_prec=lq.F16,
                            batched=batched, xref=dref)
    x = lat.to_host(dx, lq.FULL, lq.F64, 2)
    xr = lat.to_host(dref, lq.FULL, lq.F64, 2)
    for r in range(2):
        host = np.linalg.norm(x[r] - xr[r]) / np.linalg.norm(xr[r])
        say(f"  rhs {r}: ref_error {reps[r].ref_error:.3e} host {host:.3e}")
        assert abs(reps[r].ref_error - host) <= 1e-3 * host + 1e-16
        assert reps[r].ref_error <= 1e-7
    reps = lat.solve_device(dx, db, kappa, csw, tol, nrhs=2, inner_prec=lq.F16)
    assert all(r.ref_error == -1.0 for r in reps)
