"""Pins of the oracle's even-odd reduction and Krylov solvers.

The reference solution comes from a direct sparse LU of the brute-force
matrix (tests/bruteforce.py), which shares no code with the oracle.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import fields
from oracle import dirac, evenodd, solvers
from oracle.dense import dense
from tests import bruteforce


def full_matrix(u, dims, kappa, csw):
    wc = evenodd.WilsonClover(u, kappa, csw)
    h = bruteforce.hopping_matrix(u, dims)
    a = bruteforce.clover_block_matrix(wc.a.reshape(-1, 12, 12))
    return wc, (a - kappa * h).tocsc()


def test_schur_equals_dense_complement():
    dims = (2, 2, 2, 4)
    u = fields.gauge_field(dims, "haar", 101)
    wc, m = full_matrix(u, dims, 0.13, 1.0)
    par = np.repeat(bruteforce.parity_of_sites(dims), 12)
    e, o = par == 0, par == 1
    md = m.toarray()
    schur_ref = md[np.ix_(e, e)] - md[np.ix_(e, o)] @ np.linalg.solve(
        md[np.ix_(o, o)], md[np.ix_(o, e)])
    v = int(np.prod(dims))
    schur = dense(wc.schur, (v // 2, 4, 3))
    assert np.max(np.abs(schur - schur_ref)) < 1e-14
    schur_dag = dense(lambda x: wc.schur(x, dagger=True), (v // 2, 4, 3))
    assert np.max(np.abs(schur_dag - schur_ref.conj().T)) < 1e-14


def test_split_join_order():
    dims = (4, 2, 2, 2)
    psi = fields.gaussian_spinor(dims, 5)
    e, o = evenodd.split(psi, dims)
    flat = psi.reshape(-1, 4, 3)
    par = bruteforce.parity_of_sites(dims)
    assert np.array_equal(e, flat[par == 0])
    assert np.array_equal(o, flat[par == 1])
    assert np.array_equal(evenodd.join(e, o, dims), psi)


@pytest.mark.parametrize("dims,kind,kappa,csw", [
    ((2, 2, 2, 2), "haar", 0.12, 0.0),
    ((4, 4, 4, 4), "haar", 0.12, 0.0),
    ((4, 4, 4, 4), "smooth", 0.135, 1.0),
])
@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
def test_evenodd_solve_matches_direct(dims, kind, kappa, csw, method):
    u = fields.gauge_field(dims, kind, 111)
    b = fields.gaussian_spinor(dims, 112)
    wc, m = full_matrix(u, dims, kappa, csw)
    x_ref = spla.spsolve(m, b.reshape(-1))
    x, info = solvers.solve_evenodd(wc, b, tol=1e-10, method=method)
    assert info.converged and info.true_residual <= 1e-10
    # residual from the brute-force matrix, not the oracle's own operator
    res = np.linalg.norm(b.reshape(-1) - m @ x.reshape(-1)) / np.linalg.norm(b)
    assert res <= 1e-10
    cond_est = 50.0
    assert np.linalg.norm(x.reshape(-1) - x_ref) <= cond_est * 1e-10 * np.linalg.norm(x_ref)


def test_full_cgnr_and_fgmres_match_direct():
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "haar", 121)
    b = fields.gaussian_spinor(dims, 122)
    wc, m = full_matrix(u, dims, 0.12, 0.0)
    x_ref = spla.spsolve(m, b.reshape(-1))
    x1, i1 = solvers.cgnr(wc.M, wc.Mdag, b, tol=1e-10)
    x2, i2 = solvers.fgmres(wc.M, b, m=32, tol=1e-10)
    for x, info in ((x1, i1), (x2, i2)):
        assert info.converged
        assert np.linalg.norm(x.reshape(-1) - x_ref) <= 50 * 1e-10 * np.linalg.norm(x_ref)


def test_fgmres_with_varying_preconditioner_on_schur():
    """A preconditioner that changes every call (a few CG steps on the normal
    equations with a varying count) still converges under FGMRES."""
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "smooth", 131)
    b = fields.gaussian_spinor(dims, 132)
    wc = evenodd.WilsonClover(u, 0.135, 1.0)
    bhat = wc.prepare_source(b)
    calls = [0]

    def prec(v):
        calls[0] += 1
        y, _ = solvers.cgnr(wc.schur, lambda z: wc.schur(z, dagger=True), v,
                            tol=1e-30, maxiter=2 + calls[0] % 3)
        return y

    x, info = solvers.fgmres(wc.schur, bhat, precond=prec, m=16, tol=1e-10)
    assert info.converged
    assert dirac.norm(bhat - wc.schur(x)) <= 1e-10 * dirac.norm(bhat)


def test_fcg_on_normal_operator():
    dims = (4, 4, 2, 4)
    u = fields.gauge_field(dims, "smooth", 141)
    wc = evenodd.WilsonClover(u, 0.13, 1.0)
    b = wc.prepare_source(fields.gaussian_spinor(dims, 142))
    nop = lambda v: wc.schur(wc.schur(v), dagger=True)  # noqa: E731
    rhs = wc.schur(b, dagger=True)
    x, info = solvers.fcg(nop, rhs, tol=1e-10)
    assert info.converged
    assert dirac.norm(b - wc.schur(x)) <= 1e-8 * dirac.norm(b)


def test_reconstruct_solves_full_system():
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "smooth", 151)
    b = fields.gaussian_spinor(dims, 152)
    wc = evenodd.WilsonClover(u, 0.135, 1.0)
    x, info = solvers.solve_evenodd(wc, b, tol=1e-10)
    assert info.converged
    assert dirac.norm(b - wc.M(x)) <= 1e-10 * dirac.norm(b)


def test_fcg_with_varying_preconditioner_against_direct_solve():
    """The flexible branch of fcg (beta = -<q_prev, z> / <p_prev, q_prev>)
    with a preconditioner that changes at every call: a random positive
    diagonal drawn afresh each time (Hermitian positive definite, so flexible
    CG must converge).  The operator is the normal Schur operator built
    densely from the brute-force matrix, and the answer its direct solve."""
    from tests import bruteforce
    dims, kappa = (4, 4, 2, 4), 0.12
    u = fields.gauge_field(dims, "haar", 291)
    wc = evenodd.WilsonClover(u, kappa, 0.0)
    m = (bruteforce.clover_block_matrix(wc.a.reshape(-1, 12, 12))
         - kappa * bruteforce.hopping_matrix(u, dims)).toarray()
    odd = bruteforce.parity_of_sites(dims).astype(bool)
    comp = np.repeat(odd, 12)
    ie, io = np.nonzero(~comp)[0], np.nonzero(comp)[0]
    mhat = (m[np.ix_(ie, ie)]
            - m[np.ix_(ie, io)] @ np.linalg.solve(m[np.ix_(io, io)], m[np.ix_(io, ie)]))
    a = mhat.conj().T @ mhat
    rng = fields.rng(292)
    b = fields.complex_gaussian(rng, (ie.size,))
    calls = [0]

    def prec(v):
        calls[0] += 1
        d = fields.rng(300 + calls[0]).uniform(0.3, 3.0, v.size)
        return d * v

    x, info = solvers.fcg(lambda v: a @ v, b, precond=prec, tol=1e-12)
    assert info.converged
    assert calls[0] == info.iterations
    xr = np.linalg.solve(a, b)
    cond = np.linalg.cond(a)
    assert np.linalg.norm(x - xr) <= 10 * cond * 1e-12 * np.linalg.norm(xr)
    # the varying preconditioner was used: the iterates differ from plain CG
    x1, info1 = solvers.fcg(lambda v: a @ v, b, tol=1e-12)
    assert info1.iterations != info.iterations or np.linalg.norm(x1 - x) > 0


def _known_spectrum(n=300, seed=5):
    """A normal matrix with six eigenvalues of modulus 1e-3 .. 5e-3 and the
    rest of modulus 1 .. 2 (phases within +-0.3 rad), and a source."""
    rng = np.random.default_rng(seed)
    lam = (np.concatenate([np.linspace(1e-3, 5e-3, 6), rng.uniform(1, 2, n - 6)])
           * np.exp(1j * rng.uniform(-0.3, 0.3, n)))
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    a = q @ np.diag(lam) @ q.conj().T
    return a, lam, rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _arnoldi(a, v0, m):
    n = a.shape[0]
    v = np.zeros((n, m + 1), dtype=np.complex128)
    h = np.zeros((m + 1, m), dtype=np.complex128)
    v[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(m):
        w = a @ v[:, j]
        for i in range(j + 1):
            h[i, j] = np.vdot(v[:, i], w)
            w = w - h[i, j] * v[:, i]
        h[j + 1, j] = np.linalg.norm(w)
        if h[j + 1, j] > 0:
            v[:, j + 1] = w / h[j + 1, j]
    return v, h


def test_harmonic_ritz_pins():
    """(1) On an invariant Krylov space (Arnoldi run to the full dimension,
    last subdiagonal zero) harmonic Ritz values are exact eigenvalues: the k
    of smallest modulus equal those of the matrix.  (2) On a truncated
    Arnoldi matrix each pair satisfies its defining Petrov-Galerkin
    condition Hbar^dagger (Hbar g - theta [g; 0]) = 0."""
    rng = np.random.default_rng(7)
    n = 30
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    _, h = _arnoldi(a, rng.standard_normal(n) + 0j, n)
    theta, _ = solvers.harmonic_ritz(h, 5)
    ev = np.linalg.eigvals(a)
    ev = ev[np.argsort(np.abs(ev))][:5]
    for t in theta:
        assert np.min(np.abs(ev - t)) <= 1e-9 * np.abs(t)
    _, h = _arnoldi(a, rng.standard_normal(n) + 0j, 12)
    theta, g = solvers.harmonic_ritz(h, 4)
    for i in range(4):
        gi = np.concatenate([g[:, i], [0.0]])
        resid = h.conj().T @ (h @ g[:, i] - theta[i] * gi)
        assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(h) ** 2 * np.linalg.norm(g[:, i])
    # and they are the smallest-modulus solutions of that condition
    hm = h[:12, :12]
    gen = np.linalg.solve(hm.conj().T, h.conj().T @ h)
    allt = np.linalg.eigvals(gen)
    assert np.allclose(np.sort(np.abs(theta)), np.sort(np.abs(allt))[:4], rtol=1e-9)


def test_fgmres_dr_without_deflation_is_fgmres():
    """k = 0: the same iterates as restarted FGMRES(m), with a preconditioner
    that varies from call to call."""
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "smooth", 301)
    wc = evenodd.WilsonClover(u, 0.135, 1.0)
    bhat = wc.prepare_source(fields.gaussian_spinor(dims, 302))

    def make_prec():
        calls = [0]

        def prec(v):
            calls[0] += 1
            return (1.0 + 0.1 * (calls[0] % 3)) * v
        return prec

    x0, i0 = solvers.fgmres(wc.schur, bhat, precond=make_prec(), m=12, tol=1e-10)
    x1, i1 = solvers.fgmres_dr(wc.schur, bhat, precond=make_prec(), m=12, k=0, tol=1e-10)
    assert i0.iterations == i1.iterations
    assert dirac.norm(x1 - x0) <= 1e-14 * dirac.norm(x0)


def test_fgmres_dr_against_direct_solve():
    """Deflated restarts on the indefinite Schur system (kappa 0.135, clover)
    reach the direct solution of the Schur complement built densely from the
    brute-force matrix; the flexible Arnoldi relation A Z_k = V_{k+1} Hbar_k
    and the orthonormality of V_{k+1} hold after every deflated restart."""
    from tests import bruteforce
    dims, kappa, csw = (4, 4, 4, 4), 0.135, 1.0
    u = fields.gauge_field(dims, "smooth", 303)
    b = fields.gaussian_spinor(dims, 304)
    wc = evenodd.WilsonClover(u, kappa, csw)
    m = (bruteforce.clover_block_matrix(wc.a.reshape(-1, 12, 12))
         - kappa * bruteforce.hopping_matrix(u, dims)).toarray()
    odd = np.repeat(bruteforce.parity_of_sites(dims).astype(bool), 12)
    ie, io = np.nonzero(~odd)[0], np.nonzero(odd)[0]
    mhat = (m[np.ix_(ie, ie)]
            - m[np.ix_(ie, io)] @ np.linalg.solve(m[np.ix_(io, io)], m[np.ix_(io, ie)]))
    bhat = wc.prepare_source(b)
    checks = []

    def on_restart(vs, zs, hk):
        az = np.stack([wc.schur(z).reshape(-1) for z in zs], 1)
        vm = np.stack([v.reshape(-1) for v in vs], 1)
        checks.append((np.linalg.norm(az - vm @ hk) / np.linalg.norm(az),
                       np.linalg.norm(vm.conj().T @ vm - np.eye(vm.shape[1]))))

    calls = [0]

    def prec(v):  # varying: a few CG steps on the normal equations
        calls[0] += 1
        y, _ = solvers.cgnr(wc.schur, lambda z: wc.schur(z, dagger=True), v,
                            tol=1e-30, maxiter=1 + calls[0] % 3)
        return y

    x, info = solvers.fgmres_dr(wc.schur, bhat, precond=prec, m=12, k=4, tol=1e-11,
                                on_restart=on_restart)
    assert info.converged
    xr = np.linalg.solve(mhat, bhat.reshape(-1))
    cond = np.linalg.cond(mhat)
    assert np.linalg.norm(x.reshape(-1) - xr) <= 2 * cond * 1e-11 * np.linalg.norm(xr)
    assert checks, "no deflated restart happened"
    for rel_az, orth in checks:
        assert rel_az <= 1e-6 and orth <= 1e-6  # MGS in FP64, once


def test_fgmres_dr_deflates_small_eigenvalues():
    """Six eigenvalues near zero slow restarted FGMRES(20) down; keeping
    k = 6 harmonic Ritz vectors across restarts removes them (Morgan's
    argument, which the paper invokes for the low modes of the Dirac
    operator), so FGMRES-DR(20, 6) needs well under half the steps."""
    a, _, b = _known_spectrum()
    op = lambda v: a @ v  # noqa: E731
    _, plain = solvers.fgmres_dr(op, b, m=20, k=0, tol=1e-10, maxiter=5000)
    x, dr = solvers.fgmres_dr(op, b, m=20, k=6, tol=1e-10, maxiter=5000)
    assert plain.converged and dr.converged
    assert np.linalg.norm(b - a @ x) <= 1e-10 * np.linalg.norm(b)
    assert dr.iterations * 2 < plain.iterations, (dr.iterations, plain.iterations)


def _spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (q * lam) @ q.conj().T


def _galerkin(a, b, k):
    """X = K (K^H A K)^-1 K^H B over the block Krylov space
    K = span[B, A B, ..., A^(k-1) B] (orthonormalised), for X0 = 0: the
    iterate that minimises every column's A-norm error over that space."""
    blocks = [b]
    for _ in range(k - 1):
        blocks.append(a @ blocks[-1])
    kb, _ = np.linalg.qr(np.concatenate(blocks, axis=1))
    return kb @ np.linalg.solve(kb.conj().T @ a @ kb, kb.conj().T @ b)


@pytest.mark.parametrize("s,k", [(1, 5), (4, 3), (6, 2)])
def test_block_cg_iterates_are_block_krylov_projections(s, k):
    """After k iterations block CG holds the Galerkin projection of the
    solution onto the block Krylov space of dimension k s (for s = 1: CG's
    k-th iterate).  A mistake in alpha, beta or the search-block update
    leaves that space or the projection."""
    a = _spd(120, 40 + s)
    rng = np.random.default_rng(50 + s)
    b = rng.standard_normal((120, s)) + 1j * rng.standard_normal((120, s))
    x, info = solvers.block_cg(lambda v: a @ v, b.T.copy(), fixed_iterations=k)
    assert info.iterations == k
    ref = _galerkin(a, b, k)
    assert np.linalg.norm(x.T - ref) <= 1e-10 * np.linalg.norm(ref)


def test_block_cg_point_sources_against_direct_solve():
    """The 12 point sources of a propagator on the normal Schur equations of
    a 4^4 clover system (kappa 0.135): every column reaches the direct
    solution of the dense Schur complement from the brute-force matrix, in
    fewer block iterations than single-RHS CG needs for its slowest column,
    and its A-norm error never exceeds single-RHS CG's at the same
    iteration."""
    from tests import bruteforce
    dims, kappa, csw = (4, 4, 4, 4), 0.135, 1.0
    u = fields.gauge_field(dims, "smooth", 305)
    wc = evenodd.WilsonClover(u, kappa, csw)
    m = (bruteforce.clover_block_matrix(wc.a.reshape(-1, 12, 12))
         - kappa * bruteforce.hopping_matrix(u, dims)).toarray()
    odd = np.repeat(bruteforce.parity_of_sites(dims).astype(bool), 12)
    ie, io = np.nonzero(~odd)[0], np.nonzero(odd)[0]
    mhat = (m[np.ix_(ie, ie)]
            - m[np.ix_(ie, io)] @ np.linalg.solve(m[np.ix_(io, io)], m[np.ix_(io, ie)]))
    b = fields.point_sources_12(dims)
    bh = np.stack([wc.prepare_source(b[i]).reshape(-1) for i in range(12)])
    a = mhat.conj().T @ mhat
    rhs = (mhat.conj().T @ bh.T).T
    resid = lambda j, xj: np.linalg.norm(bh[j] - mhat @ xj) / np.linalg.norm(bh[j])  # noqa: E731
    x, info = solvers.block_cg(lambda v: a @ v, rhs, tol=1e-11, resid=resid)
    assert info.converged
    xr = np.linalg.solve(mhat, bh.T).T
    cond = np.linalg.cond(mhat)
    assert np.linalg.norm(x - xr) <= 2 * cond * 1e-11 * np.linalg.norm(xr)
    single = [solvers.cgnr(lambda v: mhat @ v, lambda v: mhat.conj().T @ v, bh[j],
                           tol=1e-11)[1].iterations for j in range(12)]
    assert info.iterations < max(single)
    k = 10
    xb, _ = solvers.block_cg(lambda v: a @ v, rhs, fixed_iterations=k)
    for j in range(12):
        e = xb[j] - xr[j]
        xs, _ = solvers.block_cg(lambda v: a @ v, rhs[j:j + 1], fixed_iterations=k)
        es = xs[0] - xr[j]
        assert np.vdot(e, a @ e).real <= (1 + 1e-8) * np.vdot(es, a @ es).real


def test_block_cg_dependent_columns():
    """Repeated and proportional right-hand sides make the search block rank
    deficient from the start; the dependent directions are dropped and every
    column still reaches its solution."""
    a = _spd(80, 60)
    rng = np.random.default_rng(61)
    v = rng.standard_normal(80) + 1j * rng.standard_normal(80)
    w = rng.standard_normal(80) + 1j * rng.standard_normal(80)
    b = np.stack([v, v, 2j * v, w])
    x, info = solvers.block_cg(lambda y: a @ y, b, tol=1e-11)
    assert info.converged
    for j in range(4):
        assert np.linalg.norm(a @ x[j] - b[j]) <= 1e-11 * np.linalg.norm(b[j])
    # two independent directions: at most two operator applications per iteration
    assert info.applications <= 2 * info.iterations
