"""Schwarz alternating procedure (SAP) preconditioner and flexible GCR, FP64
(oracle; test infrastructure only).

Paper, section 5 (its SAP-FGCR solver):
* The lattice is cut into non-overlapping blocks, coloured like a
  checkerboard.
* One SAP cycle solves the Wilson-Dirac equation on every block of one
  colour, then updates the residual, then solves on the blocks of the other
  colour with the updated residual as source, then updates the residual again.
* Block solves take a fixed number of minimal-residual (MR) iterations, with
  Dirichlet boundary conditions (hops that leave a block are dropped).
* SAP preconditions a flexible GCR (FGCR, equivalent to FGMRES). FGCR is
  restarted, and the residual is recomputed in double precision at each
  restart.

The paper prints no formulas for either, so these readings are taken:
* Blocks have extents B dividing the lattice, with an even number of blocks
  (at least 2) per direction. The colouring is then consistent across the
  periodic boundary, and two blocks of one colour never share a face.
* A block's colour is the sum of its block coordinates mod 2. Colour 0 is
  solved first.
* The block solver is MR on the block restriction M_b of M itself. Each
  iteration takes q = M_b rho, alpha = <q, rho> / <q, q> (0 if q = 0),
  delta += alpha rho, rho -= alpha q, starting from delta = 0 and rho = the
  residual on the block.
* Optionally (the refinement the paper's performance model counts as a factor
  (n_it + 1) / n_it), the blocks are even-odd reduced. MR then runs on the
  block Schur operator, and the odd sites are reconstructed (mr_blocks_eo).
* The preconditioner runs ncy cycles on the source eta from psi = 0. After
  each half cycle the residual is eta - M psi. This equals the paper's update
  on the solved blocks and on the borders of the others.
* FGCR is right-preconditioned GCR with the preconditioner applied afresh at
  every step (so it may vary). The M z vectors are orthonormalised by
  modified Gram-Schmidt, and the z vectors are transformed with them. The
  recursion restarts every m steps, with the residual recomputed from M.

Pins (tests/test_oracle_sap.py):
* the block MR against dense MR on block submatrices of the brute-force
  sparse matrix, and the even-odd block MR against dense MR on the Schur
  complement of those submatrices;
* the Schwarz property: after a half cycle with converged block solves, the
  residual vanishes on the solved blocks;
* the multiplicative structure: one cycle with converged block solves equals
  the dense block Gauss-Seidel sweep psi_0 = M_00^-1 eta_0,
  psi_1 = M_11^-1 (eta_1 - M_10 psi_0), and several cycles of few MR steps
  equal the procedure run block by block on dense submatrices (an additive
  variant fails both);
* M = 1 gives K = 1 exactly;
* FGCR against a direct sparse solve.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import clover as _clover
from oracle import dirac


def block_layout(dims, block):
    """Block id and colour of every site, as arrays of the lattice shape
    (t, z, y, x).  dims and block are (x, y, z, t) extents."""
    for d, b in zip(dims, block):
        if b < 1 or d % b != 0 or (d // b) % 2 != 0:
            raise ValueError("each block extent must divide the lattice extent an even "
                             "number of times")
    nb = [d // b for d, b in zip(dims, block)]
    lx, ly, lz, lt = dims
    x = np.arange(lx) // block[0]
    y = np.arange(ly) // block[1]
    z = np.arange(lz) // block[2]
    t = np.arange(lt) // block[3]
    bt, bz, by, bx = np.meshgrid(t, z, y, x, indexing="ij")
    bid = ((bt * nb[2] + bz) * nb[1] + by) * nb[0] + bx
    colour = (bx + by + bz + bt) % 2
    return bid, colour


def _block_sums(v, bid, nblocks):
    """Per-block sums of a complex site field v (lattice shape)."""
    flat = bid.reshape(-1)
    return (np.bincount(flat, weights=v.real.reshape(-1), minlength=nblocks)
            + 1j * np.bincount(flat, weights=v.imag.reshape(-1), minlength=nblocks))


def mr_blocks(op, r, mask, bid, nblocks, nmr):
    """nmr MR iterations on every block of a colour at once, from zero.

    op: the full-lattice operator M; mask: sites of the colour (lattice
    shape, bool); the block operator M_b v = (M v)|_b for v supported on the
    block, so for a whole colour op_b v = mask * M(mask * v).  Returns delta
    (zero off the colour)."""
    m = mask[..., None, None]
    rho = np.where(m, r, 0)
    delta = np.zeros_like(r)
    for _ in range(nmr):
        q = np.where(m, op(rho), 0)
        qr = _block_sums(np.sum(np.conj(q) * rho, axis=(-2, -1)), bid, nblocks)
        qq = _block_sums(np.sum(np.abs(q) ** 2, axis=(-2, -1)), bid, nblocks).real
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1), 0)
        a = alpha[bid][..., None, None]
        delta = delta + a * rho
        rho = rho - a * q
    return delta


def mr_blocks_eo(wc, r, mask, bid, nblocks, nmr, odd):
    """nmr MR steps on the even-odd reduced block operator of every block of
    a colour (the refinement the paper's performance model counts).

    With H_b the block-restricted hopping term (Dirichlet), the block system
    M_b d = r splits into even and odd sites; MR runs on
        Mhat_b d_e = A_ee d_e - kappa^2 H_eo^b A_oo^-1 H_oe^b d_e
    with source r_e + kappa H_eo^b A_oo^-1 r_o, from d_e = 0, and
        d_o = A_oo^-1 (r_o + kappa H_oe^b d_e).
    wc: the WilsonClover operator (A, A^-1, H); odd: odd-site mask (lattice
    shape).  Returns d (zero off the colour)."""
    k = wc.kappa
    m = mask[..., None, None]
    me = (mask & ~odd)[..., None, None]
    mo = (mask & odd)[..., None, None]

    def hb(v):  # block hopping term, restricted to the colour's blocks
        return np.where(m, wc.hop(np.where(m, v, 0)), 0)

    def ainv_o(v):
        return np.where(mo, _clover.apply_site_matrix(wc.ainv, v), 0)

    def a_e(v):
        return np.where(me, _clover.apply_site_matrix(wc.a, v), 0)

    re_ = np.where(me, r, 0)
    ro = np.where(mo, r, 0)
    rho = re_ + k * np.where(me, hb(ainv_o(ro)), 0)
    de = np.zeros_like(r)
    for _ in range(nmr):
        q = a_e(rho) - k * k * np.where(me, hb(ainv_o(hb(rho))), 0)
        qr = _block_sums(np.sum(np.conj(q) * rho, axis=(-2, -1)), bid, nblocks)
        qq = _block_sums(np.sum(np.abs(q) ** 2, axis=(-2, -1)), bid, nblocks).real
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1), 0)
        a = alpha[bid][..., None, None]
        de = de + a * rho
        rho = rho - a * q
    do = ainv_o(ro + k * np.where(mo, hb(de), 0))
    return de + do


def sap(op, eta, dims, block, ncy, nmr, wc=None):
    """psi = K eta: ncy SAP cycles from psi = 0 (colour 0 first).  With wc
    (the WilsonClover operator) the blocks are solved by MR on their even-odd
    reduced operator (mr_blocks_eo), else by MR on M_b itself."""
    bid, colour = block_layout(dims, block)
    nblocks = int(bid.max()) + 1
    if wc is not None:
        from oracle import evenodd
        odd = evenodd.odd_mask(dims)
    psi = np.zeros_like(eta)
    r = eta.copy()
    for _ in range(ncy):
        for c in (0, 1):
            if wc is None:
                psi = psi + mr_blocks(op, r, colour == c, bid, nblocks, nmr)
            else:
                psi = psi + mr_blocks_eo(wc, r, colour == c, bid, nblocks, nmr, odd)
            r = eta - op(psi)
    return psi


@dataclass
class Info:
    iterations: int = 0
    restarts: int = 0
    converged: bool = False
    residual: float = np.inf


def fgcr(op, b, precond, m=16, tol=1e-10, maxiter=10000, x0=None):
    """Flexible right-preconditioned GCR, restarted every m steps; stops on
    the true residual ||b - op x|| / ||b|| <= tol."""
    info = Info()
    bn = dirac.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        info.converged, info.residual = True, 0.0
        return np.zeros_like(b), info
    while True:
        r = b - op(x)
        info.residual = dirac.norm(r) / bn
        if info.residual <= tol:
            info.converged = True
            return x, info
        if info.iterations >= maxiter:
            return x, info
        info.restarts += 1
        zs, ws = [], []
        for _ in range(m):
            z = precond(r)
            w = op(z)
            for zj, wj in zip(zs, ws):
                beta = dirac.inner(wj, w)
                w = w - beta * wj
                z = z - beta * zj
            wn = dirac.norm(w)
            if wn == 0.0:
                break
            w, z = w / wn, z / wn
            alpha = dirac.inner(w, r)
            x = x + alpha * z
            r = r - alpha * w
            zs.append(z)
            ws.append(w)
            info.iterations += 1
            if dirac.norm(r) <= 0.1 * tol * bn or info.iterations >= maxiter:
                break
