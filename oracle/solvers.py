"""Krylov solvers in FP64 (oracle, test infrastructure).

Paper: section 3 gives the problem M phi = b or M^dagger M phi = b; section 5
names CG on the normal operator (exploiting its Hermiticity and positive
definiteness), CG on the even-odd Schur equation, FGCR (mathematically equal
to FGMRES, tolerant of a varying preconditioner, restarted) and mixed
precision by iterative refinement (residual recomputed in double precision
at each restart, single-precision correction added to the double solution).
Recurrences are not printed in the paper; the textbook forms are used:

* cgnr:     Hestenes-Stiefel CG on A^dagger A x = A^dagger b from x = 0;
* bicgstab: van der Vorst's BiCGStab, restarting the shadow residual when
            rho breaks down;
* fgmres:   right-preconditioned restarted FGMRES(m), modified Gram-Schmidt
            Arnoldi, true residual recomputed at every restart;
* fcg:      flexible (Notay) preconditioned CG on a Hermitian positive
            definite operator;
* fgmres_dr: FGMRES with deflated restarting (section 7 of the paper, after
            Morgan's GMRES-DR): k harmonic Ritz vectors of smallest modulus
            are carried across each restart;
* block_cg: O'Leary's block CG for several right-hand sides sharing one
            block Krylov space (breakdown-free form with a rank-revealing
            search block).

Every solver stops on the true residual ||b - A x|| / ||b|| <= tol computed
from the operator, never on a recurrence value alone.  Functions take
callables on NumPy arrays of any shape.

Pins (CPU tests): dense LU solutions on 2^4 and 4^4 lattices; fcg with a
preconditioner that changes at every call against the direct solve of the
dense normal Schur operator; fgmres_dr against the dense Schur solve, equal
to fgmres for k = 0, with the flexible Arnoldi relation after each deflated
restart, and deflating a known set of small eigenvalues; harmonic Ritz
values exact on an invariant subspace and satisfying their Petrov-Galerkin
condition; block_cg's iterates equal to the Galerkin projection onto the
block Krylov space built densely, its 12 point-source solutions equal to the
dense Schur solve, its A-norm errors never above single-RHS CG's, and
dependent right-hand sides.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .dirac import inner, norm


@dataclass
class SolveInfo:
    iterations: int = 0
    converged: bool = False
    true_residual: float = float("nan")
    history: list = field(default_factory=list)


def cgnr(op, opdag, b, tol=1e-10, maxiter=10000, x0=None):
    """CG on the normal equations A^dagger A x = A^dagger b."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.true_residual = True, 0.0
        return x, info
    r = opdag(b - op(x))
    p = r.copy()
    rr = inner(r, r).real
    for k in range(maxiter):
        q = op(p)
        alpha = rr / inner(q, q).real
        x += alpha * p
        r -= alpha * opdag(q)
        rr_new = inner(r, r).real
        info.iterations = k + 1
        info.history.append(np.sqrt(rr_new))
        # the normal-equation residual bounds the true one loosely; check the
        # true residual when the recurrence suggests we may be done
        if np.sqrt(rr_new) <= tol * bnorm * 1e-2 or k % 25 == 24:
            res = norm(b - op(x)) / bnorm
            if res <= tol:
                info.converged, info.true_residual = True, res
                return x, info
        p = r + (rr_new / rr) * p
        rr = rr_new
    info.true_residual = norm(b - op(x)) / bnorm
    info.converged = info.true_residual <= tol
    return x, info


def bicgstab(op, b, tol=1e-10, maxiter=10000, x0=None):
    """van der Vorst BiCGStab on A x = b."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.true_residual = True, 0.0
        return x, info
    r = b - op(x)
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for k in range(maxiter):
        rho_new = inner(rhat, r)
        if abs(rho_new) < 1e-30 * norm(r) * norm(rhat):
            rhat = r.copy()
            rho_new = inner(rhat, r)
            p = np.zeros_like(b)
            v = np.zeros_like(b)
            rho = alpha = omega = 1.0 + 0j
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = op(p)
        alpha = rho_new / inner(rhat, v)
        s = r - alpha * v
        t = op(s)
        omega = inner(t, s) / inner(t, t)
        x += alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        info.iterations = k + 1
        rn = norm(r)
        info.history.append(rn)
        if rn <= tol * bnorm * 0.5 or k % 25 == 24:
            res = norm(b - op(x)) / bnorm
            if res <= tol:
                info.converged, info.true_residual = True, res
                return x, info
    info.true_residual = norm(b - op(x)) / bnorm
    info.converged = info.true_residual <= tol
    return x, info


def fgmres(op, b, precond=None, m=32, tol=1e-10, maxiter=10000, x0=None):
    """Restarted right-preconditioned flexible GMRES(m)."""
    if precond is None:
        precond = lambda v: v  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.true_residual = True, 0.0
        return x, info
    total = 0
    while total < maxiter:
        r = b - op(x)
        beta = norm(r)
        info.true_residual = beta / bnorm
        info.history.append(beta)
        if info.true_residual <= tol:
            info.converged = True
            break
        vs = [r / beta]
        zs = []
        h = np.zeros((m + 1, m), dtype=np.complex128)
        j_used = 0
        for j in range(m):
            z = precond(vs[j])
            zs.append(z)
            w = op(z)
            for i in range(j + 1):
                h[i, j] = inner(vs[i], w)
                w = w - h[i, j] * vs[i]
            h[j + 1, j] = norm(w)
            j_used = j + 1
            total += 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(h[: j + 2, : j + 1], e1, rcond=None)
            est = norm(e1 - h[: j + 2, : j + 1] @ y)
            if h[j + 1, j].real == 0.0 or est <= 0.5 * tol * bnorm or total >= maxiter:
                break
            vs.append(w / h[j + 1, j])
        e1 = np.zeros(j_used + 1, dtype=np.complex128)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(h[: j_used + 1, :j_used], e1, rcond=None)
        for i in range(j_used):
            x = x + y[i] * zs[i]
    info.iterations = total
    info.true_residual = norm(b - op(x)) / bnorm
    info.converged = info.true_residual <= tol
    return x, info


def fcg(op, b, precond=None, tol=1e-10, maxiter=10000, x0=None):
    """Flexible preconditioned CG (Notay) for Hermitian positive definite op."""
    if precond is None:
        precond = lambda v: v  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.true_residual = True, 0.0
        return x, info
    r = b - op(x)
    p_prev = q_prev = None
    pq_prev = 1.0
    for k in range(maxiter):
        z = precond(r)
        if p_prev is None:
            p = z
        else:
            p = z - (inner(q_prev, z) / pq_prev) * p_prev
        q = op(p)
        pq = inner(p, q).real
        alpha = inner(p, r) / pq
        x = x + alpha * p
        r = r - alpha * q
        p_prev, q_prev, pq_prev = p, q, pq
        info.iterations = k + 1
        info.history.append(norm(r))
        if norm(r) <= 0.5 * tol * bnorm or k % 25 == 24:
            res = norm(b - op(x)) / bnorm
            if res <= tol:
                info.converged, info.true_residual = True, res
                return x, info
    info.true_residual = norm(b - op(x)) / bnorm
    info.converged = info.true_residual <= tol
    return x, info


def solve_evenodd(wc, b_full, tol=1e-10, method="cgnr", maxiter=20000):
    """Solve M x = b through the Schur system; stop on the full-system residual.

    Iterate on Mhat x_e = bhat_e to 0.5*tol, reconstruct x_o and check
    ||b - M x|| / ||b|| <= tol; if not met, continue from x_e with the
    Schur tolerance halved (at most three times).
    """
    bhat = wc.prepare_source(b_full)
    op = wc.schur
    opdag = lambda v: wc.schur(v, dagger=True)  # noqa: E731
    x_e = None
    t = 0.5 * tol
    iters = 0
    for _ in range(4):
        if method == "cgnr":
            x_e, info = cgnr(op, opdag, bhat, t, maxiter, x_e)
        elif method == "bicgstab":
            x_e, info = bicgstab(op, bhat, t, maxiter, x_e)
        else:
            raise ValueError(method)
        iters += info.iterations
        x = wc.reconstruct(x_e, b_full)
        res = norm(b_full - wc.M(x)) / norm(b_full)
        if res <= tol:
            break
        t *= 0.5
    return x, SolveInfo(iterations=iters, converged=res <= tol, true_residual=res)


def harmonic_ritz(hbar, k):
    """The k harmonic Ritz pairs of smallest modulus from an (j+1) x j
    upper Hessenberg Arnoldi matrix hbar (A Z_j = V_{j+1} hbar): the
    eigenpairs of H_j + |h_{j+1,j}|^2 f e_j^dagger with f = H_j^-dagger e_j
    (H_j the square top of hbar).  Returns (theta[k], G[j, k])."""
    j = hbar.shape[1]
    hm = hbar[:j, :j]
    ej = np.zeros(j, dtype=np.complex128)
    ej[-1] = 1.0
    f = np.linalg.solve(hm.conj().T, ej)
    g = hm + abs(hbar[j, j - 1]) ** 2 * np.outer(f, ej)
    theta, vecs = np.linalg.eig(g)
    order = np.argsort(np.abs(theta))[:k]
    return theta[order], vecs[:, order]


def fgmres_dr(op, b, precond=None, m=32, k=0, tol=1e-10, maxiter=10000, x0=None,
              on_restart=None):
    """Right-preconditioned flexible GMRES with deflated restarting (Morgan's
    GMRES-DR with the flexible Arnoldi relation A Z_m = V_{m+1} Hbar_m).

    m is the largest subspace dimension, including the k deflated vectors.
    A cycle runs the Arnoldi process (modified Gram-Schmidt) to m columns,
    solves the small least-squares problem min |c - Hbar y| and updates
    x += Z y.  Without deflation (k = 0, or after a cycle that stopped early)
    the next cycle starts afresh from the residual.  With deflation:
      1. the k harmonic Ritz vectors g_i of smallest |theta| (harmonic_ritz);
      2. P_{k+1}: orthonormalise [g_1 .. g_k] (a zero appended to each) and
         then the least-squares residual s = c - Hbar y;
      3. V <- V_{m+1} P_{k+1}, Z <- Z_m P_k (P_k = the top m rows of the
         first k columns), Hbar <- P_{k+1}^dagger Hbar_m P_k, c <- P_{k+1}^dagger s;
      4. the Arnoldi process continues from column k.
    The stopping test is the true residual |b - op x| / |b| <= tol at the end
    of every cycle.  on_restart(V, Z, hbar), if given, sees the basis after
    each deflated restart (for tests of A Z_k = V_{k+1} Hbar_k)."""
    if precond is None:
        precond = lambda v: v  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.true_residual = True, 0.0
        return x, info
    total = 0
    vs = zs = None
    h = c = None
    j0 = 0
    while True:
        if j0 == 0:  # fresh start from the residual
            r = b - op(x)
            beta = norm(r)
            vs, zs = [r / beta], []
            h = np.zeros((m + 1, m), dtype=np.complex128)
            c = np.zeros(m + 1, dtype=np.complex128)
            c[0] = beta
        jend = j0
        broke = False
        for j in range(j0, m):
            z = precond(vs[j])
            zs.append(z)
            w = op(z)
            for i in range(j + 1):
                h[i, j] = inner(vs[i], w)
                w = w - h[i, j] * vs[i]
            h[j + 1, j] = norm(w)
            jend = j + 1
            total += 1
            y, *_ = np.linalg.lstsq(h[: j + 2, : j + 1], c[: j + 2], rcond=None)
            est = norm(c[: j + 2] - h[: j + 2, : j + 1] @ y)
            if h[j + 1, j].real == 0.0 or est <= 0.5 * tol * bnorm or total >= maxiter:
                broke = True
                break
            vs.append(w / h[j + 1, j])
        hb = h[: jend + 1, :jend]
        y, *_ = np.linalg.lstsq(hb, c[: jend + 1], rcond=None)
        for i in range(jend):
            x = x + y[i] * zs[i]
        res = norm(b - op(x)) / bnorm
        info.history.append(res)
        info.true_residual = res
        if res <= tol:
            info.converged = True
            break
        if total >= maxiter:
            break
        if k == 0 or broke or jend < m:
            j0 = 0
            continue
        # deflated restart
        s = c[: m + 1] - hb @ y
        _, g = harmonic_ritz(hb, k)
        p = np.zeros((m + 1, k + 1), dtype=np.complex128)
        p[:m, :k] = g
        p[:, k] = s
        p, _ = np.linalg.qr(p)
        pk = p[:m, :k]
        vs = [sum(p[i, a] * vs[i] for i in range(m + 1)) for a in range(k + 1)]
        zs = [sum(pk[i, a] * zs[i] for i in range(m)) for a in range(k)]
        hk = p.conj().T @ hb @ pk
        c_new = p.conj().T @ s
        h = np.zeros((m + 1, m), dtype=np.complex128)
        h[: k + 1, :k] = hk
        c = np.zeros(m + 1, dtype=np.complex128)
        c[: k + 1] = c_new
        j0 = k
        if on_restart is not None:
            on_restart(vs, zs, hk)
    info.iterations = total
    return x, info


def _orth(w, drop_tol):
    """Orthonormal basis of the column space of w (N x s), dropping the
    directions whose singular value is below drop_tol."""
    u, sv, _ = np.linalg.svd(w, full_matrices=False)
    return u[:, sv > drop_tol]


def block_cg(op, b, tol=1e-10, maxiter=10000, x0=None, drop_tol=1e-13, resid=None,
             fixed_iterations=None):
    """Block CG for s right-hand sides of a Hermitian positive definite
    operator (O'Leary's block conjugate gradient, in the breakdown-free form
    that keeps an orthonormal, rank-revealing search block).

    b: (s, ...) stack of right-hand sides; op acts on one field.  The columns
    are first scaled to unit norm (the block Krylov space does not change).
    With R = B - A X and P = orth(R):
        Q = A P,  alpha = (P^H Q)^-1 P^H R,  X += P alpha,  R -= Q alpha,
        beta = -(P^H Q)^-1 Q^H R,  P = orth(R + P beta),
    where orth drops directions of singular value below drop_tol (in units of
    the scaled right-hand sides): directions that became dependent, and those
    of columns already solved to that level.  Each iteration applies op to
    the columns of P (at most s).  Stops when resid(j, x_j) <= tol for every
    column (default |b_j - op x_j| / |b_j|), checked every iteration, or after
    fixed_iterations iterations when given."""
    s = b.shape[0]
    shape = b.shape[1:]
    bm = b.reshape(s, -1).T  # N x s
    scale = np.linalg.norm(bm, axis=0)
    scale[scale == 0.0] = 1.0
    bs = bm / scale
    x = np.zeros_like(bs) if x0 is None else x0.reshape(s, -1).T / scale

    def apply(p):
        return np.stack([op(p[:, j].reshape(shape)).reshape(-1) for j in range(p.shape[1])], 1)

    if resid is None:
        bn = np.linalg.norm(bm, axis=0)

        def resid(j, xj):
            return norm(b[j] - op(xj)) / bn[j] if bn[j] > 0 else 0.0

    info = SolveInfo()
    r = bs - apply(x) if x0 is not None else bs.copy()
    p = _orth(r, drop_tol)
    applications = 0
    for k in range(maxiter):
        if p.shape[1] == 0:
            break
        q = apply(p)
        applications += p.shape[1]
        pq = p.conj().T @ q
        alpha = np.linalg.solve(pq, p.conj().T @ r)
        x = x + p @ alpha
        r = r - q @ alpha
        info.iterations = k + 1
        if fixed_iterations is not None:
            if k + 1 >= fixed_iterations:
                break
        else:
            res = [resid(j, (x[:, j] * scale[j]).reshape(shape)) for j in range(s)]
            info.history.append(max(res))
            if max(res) <= tol:
                info.converged = True
                info.true_residual = max(res)
                break
        beta = -np.linalg.solve(pq, q.conj().T @ r)
        p = _orth(r + p @ beta, drop_tol)
    info.applications = applications
    return (x * scale).T.reshape(b.shape), info
