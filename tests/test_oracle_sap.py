"""Pins of the SAP preconditioner and FGCR oracle (oracle/sap.py).

* Block MR is checked against dense MR on submatrices of the brute-force
  sparse matrix. Restricting the full matrix to one block's rows and columns
  is exactly the Dirichlet block operator, written independently of the
  oracle's masked stencil.
* The Schwarz property: with converged block solves, a half cycle leaves no
  residual on the blocks it solved.
* M = 1 (kappa = 0, no clover term) gives K = 1 exactly.
* FGCR with SAP reaches the direct sparse solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import fields
from oracle import dirac, evenodd, sap
from tests import bruteforce


def full_matrix(u, dims, kappa, csw):
    wc = evenodd.WilsonClover(u, kappa, csw)
    h = bruteforce.hopping_matrix(u, dims)
    a = bruteforce.clover_block_matrix(wc.a.reshape(-1, 12, 12))
    return wc, (a - kappa * h).tocsr()


def test_block_layout_rejects_odd_block_counts():
    with pytest.raises(ValueError):
        sap.block_layout((4, 4, 4, 6), (2, 2, 2, 2))  # 3 blocks in t
    with pytest.raises(ValueError):
        sap.block_layout((4, 4, 4, 4), (4, 2, 2, 2))  # 1 block in x
    bid, colour = sap.block_layout((4, 4, 4, 8), (2, 2, 2, 2))
    assert bid.max() + 1 == 2 * 2 * 2 * 4
    # every face neighbour of a site in another block has the other colour
    for mu in range(4):
        axis = 3 - mu
        other = np.roll(bid, 1, axis=axis) != bid
        assert np.all(np.roll(colour, 1, axis=axis)[other] != colour[other])


@pytest.mark.parametrize("nmr", [1, 4])
def test_block_mr_against_dense_blocks(nmr):
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    u = fields.gauge_field(dims, "smooth", 211)
    r = fields.gaussian_spinor(dims, 212)
    wc, mat = full_matrix(u, dims, 0.13, 1.0)
    bid, colour = sap.block_layout(dims, block)
    nblocks = int(bid.max()) + 1
    for c in (0, 1):
        got = sap.mr_blocks(wc.M, r, colour == c, bid, nblocks, nmr).reshape(-1)
        flat_r = r.reshape(-1)
        ref = np.zeros_like(flat_r)
        for b in range(nblocks):
            sites = np.nonzero(bid.reshape(-1) == b)[0]
            if colour.reshape(-1)[sites[0]] != c:
                continue
            idx = (sites[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)
            mb = mat[idx][:, idx].toarray()
            rho = flat_r[idx].copy()
            delta = np.zeros_like(rho)
            for _ in range(nmr):
                q = mb @ rho
                alpha = np.vdot(q, rho) / np.vdot(q, q)
                delta += alpha * rho
                rho -= alpha * q
            ref[idx] = delta
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_schwarz_property_with_converged_blocks():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    u = fields.gauge_field(dims, "smooth", 213)
    eta = fields.gaussian_spinor(dims, 214)
    wc = evenodd.WilsonClover(u, 0.12, 1.0)
    bid, colour = sap.block_layout(dims, block)
    nblocks = int(bid.max()) + 1
    mask = colour == 0
    psi = sap.mr_blocks(wc.M, eta, mask, bid, nblocks, 200)
    r = eta - wc.M(psi)
    assert dirac.norm(r[mask]) <= 1e-10 * dirac.norm(eta[mask])
    assert dirac.norm(r[~mask]) > 0.1 * dirac.norm(eta[~mask])


def test_identity_operator_gives_identity():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    u = fields.gauge_field(dims, "haar", 215)
    eta = fields.gaussian_spinor(dims, 216)
    wc = evenodd.WilsonClover(u, 0.0, 0.0)
    psi = sap.sap(wc.M, eta, dims, block, ncy=3, nmr=2)
    assert np.array_equal(psi, eta)


def test_fgcr_with_sap_matches_direct_solve():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    kappa, csw = 0.13, 1.0
    u = fields.gauge_field(dims, "smooth", 217)
    b = fields.gaussian_spinor(dims, 218)
    wc, mat = full_matrix(u, dims, kappa, csw)
    x, info = sap.fgcr(wc.M, b, lambda v: sap.sap(wc.M, v, dims, block, 2, 4), m=8, tol=1e-10)
    assert info.converged
    xr = spla.spsolve(mat.tocsc(), b.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - xr) <= 1e-8 * np.linalg.norm(xr)
    # the preconditioner pays: fewer steps than plain GCR
    _, plain = sap.fgcr(wc.M, b, lambda v: v, m=8, tol=1e-10)
    assert info.iterations < plain.iterations


@pytest.mark.parametrize("nmr", [1, 3])
def test_even_odd_block_mr_against_dense_schur(nmr):
    """MR on the even-odd reduced block operator, against dense MR on the
    Schur complement of each block submatrix of the brute-force matrix, with
    the odd sites reconstructed densely."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    kappa = 0.13
    u = fields.gauge_field(dims, "smooth", 219)
    r = fields.gaussian_spinor(dims, 220)
    wc, mat = full_matrix(u, dims, kappa, 1.0)
    bid, colour = sap.block_layout(dims, block)
    nblocks = int(bid.max()) + 1
    odd = evenodd.odd_mask(dims).reshape(-1)
    for c in (0, 1):
        got = sap.mr_blocks_eo(wc, r, colour == c, bid, nblocks, nmr,
                               evenodd.odd_mask(dims)).reshape(-1)
        flat_r = r.reshape(-1)
        ref = np.zeros_like(flat_r)
        for b in range(nblocks):
            sites = np.nonzero(bid.reshape(-1) == b)[0]
            if colour.reshape(-1)[sites[0]] != c:
                continue
            se, so = sites[~odd[sites]], sites[odd[sites]]
            ie = (se[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)
            io = (so[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)
            mee = mat[ie][:, ie].toarray()
            meo = mat[ie][:, io].toarray()
            moe = mat[io][:, ie].toarray()
            moo = mat[io][:, io].toarray()
            mooi = np.linalg.inv(moo)
            schur = mee - meo @ mooi @ moe
            rho = flat_r[ie] - meo @ mooi @ flat_r[io]
            de = np.zeros_like(rho)
            for _ in range(nmr):
                q = schur @ rho
                alpha = np.vdot(q, rho) / np.vdot(q, q)
                de += alpha * rho
                rho -= alpha * q
            ref[ie] = de
            ref[io] = mooi @ (flat_r[io] - moe @ de)
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def _colour_blocks(dims, block, colour_id):
    """Per block of the colour: its sites' 12-component matrix indices."""
    bid, colour = sap.block_layout(dims, block)
    out = []
    for b in range(int(bid.max()) + 1):
        sites = np.nonzero(bid.reshape(-1) == b)[0]
        if colour.reshape(-1)[sites[0]] == colour_id:
            out.append((sites[:, None] * 12 + np.arange(12)[None, :]).reshape(-1))
    return out


def _dense_sap(mat, eta, dims, block, ncy, nmr):
    """The Schwarz alternating procedure written on the brute-force matrix:
    per cycle and colour (0 first), dense MR (nmr steps, or a direct solve
    when nmr is None) on each block submatrix with the current residual as
    source, then the residual recomputed with the whole matrix."""
    m = mat.toarray()
    eta = eta.reshape(-1)
    psi = np.zeros_like(eta)
    r = eta.copy()
    for _ in range(ncy):
        for c in (0, 1):
            for idx in _colour_blocks(dims, block, c):
                mb = m[np.ix_(idx, idx)]
                if nmr is None:
                    psi[idx] += np.linalg.solve(mb, r[idx])
                    continue
                rho = r[idx].copy()
                for _ in range(nmr):
                    q = mb @ rho
                    alpha = np.vdot(q, rho) / np.vdot(q, q)
                    psi[idx] += alpha * rho
                    rho -= alpha * q
            r = eta - m @ psi
    return psi


def _additive_sap(op, eta, dims, block, ncy, nmr):
    """A plausible mistake: both colours solved against the same residual
    (additive Schwarz) instead of the second against the residual the first
    left.  Used only to show that the pins below tell the two apart."""
    bid, colour = sap.block_layout(dims, block)
    nblocks = int(bid.max()) + 1
    psi = np.zeros_like(eta)
    r = eta.copy()
    for _ in range(ncy):
        d0 = sap.mr_blocks(op, r, colour == 0, bid, nblocks, nmr)
        d1 = sap.mr_blocks(op, r, colour == 1, bid, nblocks, nmr)
        psi = psi + d0 + d1
        r = eta - op(psi)
    return psi


def test_sap_cycle_is_block_gauss_seidel():
    """One cycle with converged block solves is one multiplicative block
    Gauss-Seidel sweep over the two colours (section 5: the second colour is
    solved with the residual the first left):
        psi_0 = M_00^-1 eta_0,   psi_1 = M_11^-1 (eta_1 - M_10 psi_0),
    with M_cc block diagonal over the blocks of colour c (two blocks of one
    colour never touch).  Built here from the brute-force matrix by dense
    solves; an additive variant misses it by far."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    u = fields.gauge_field(dims, "smooth", 281)
    eta = fields.gaussian_spinor(dims, 282)
    wc, mat = full_matrix(u, dims, 0.12, 1.0)
    m = mat.toarray()
    e = eta.reshape(-1)
    idx0 = np.concatenate(_colour_blocks(dims, block, 0))
    idx1 = np.concatenate(_colour_blocks(dims, block, 1))
    psi0 = np.linalg.solve(m[np.ix_(idx0, idx0)], e[idx0])
    psi1 = np.linalg.solve(m[np.ix_(idx1, idx1)], e[idx1] - m[np.ix_(idx1, idx0)] @ psi0)
    ref = np.zeros_like(e)
    ref[idx0], ref[idx1] = psi0, psi1
    # the block-by-block dense procedure agrees with the two-colour closed form
    dense = _dense_sap(mat, eta, dims, block, 1, None)
    assert np.linalg.norm(dense - ref) <= 1e-12 * np.linalg.norm(ref)
    got = sap.sap(wc.M, eta, dims, block, ncy=1, nmr=300).reshape(-1)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)
    add = _additive_sap(wc.M, eta, dims, block, ncy=1, nmr=300).reshape(-1)
    assert np.linalg.norm(add - ref) >= 1e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("ncy,nmr", [(2, 2), (3, 1)])
def test_sap_cycles_against_dense_block_mr(ncy, nmr):
    """Several cycles of few MR steps, against the same procedure run block by
    block with dense submatrices of the brute-force matrix; the additive
    variant fails the same comparison."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    u = fields.gauge_field(dims, "smooth", 283)
    eta = fields.gaussian_spinor(dims, 284)
    wc, mat = full_matrix(u, dims, 0.13, 1.0)
    ref = _dense_sap(mat, eta, dims, block, ncy, nmr)
    got = sap.sap(wc.M, eta, dims, block, ncy=ncy, nmr=nmr).reshape(-1)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    add = _additive_sap(wc.M, eta, dims, block, ncy=ncy, nmr=nmr).reshape(-1)
    assert np.linalg.norm(add - ref) >= 1e-2 * np.linalg.norm(ref)
