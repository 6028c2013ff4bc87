"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws random numbers and shapes them into lattice fields.
None of the method's arithmetic (hopping term, clover term, solvers) lives
here: both the CPU oracle and the HIP library receive these arrays as plain
inputs.

Host canonical layouts (the C-ABI uses the same ones):

* lattice dimensions are given as ``dims = (Lx, Ly, Lz, Lt)``, all even;
* a full-lattice array has leading axes ``(Lt, Lz, Ly, Lx)`` so that its
  flattened site index is ``i = ((x3*Lz + x2)*Ly + x1)*Lx + x0``;
* gauge field ``U[..., mu, a, b]`` complex128, ``U_mu(x)`` the link x -> x+mu;
* spinor ``psi[..., s, a]`` complex128 (spin major, colour minor);
* a half-lattice array lists the sites of one parity in increasing ``i``.

The paper's workloads are physical gauge ensembles (Chroma and BQCD runs,
section 6 and 7); these generators stand in for them with Haar-random or
smooth SU(3) fields of the same shapes.
"""
from __future__ import annotations

import numpy as np

# Seeds per workload: gauge 1000+k, source 2000+k, gauge transform 3000+k for
# workload k; learned-preconditioner training field 4000, validation field
# 4001, training sources 5000+i.
SEED_GAUGE = 1000
SEED_SOURCE = 2000
SEED_TRANSFORM = 3000
SEED_TRAIN_FIELD = 4000
SEED_VALID_FIELD = 4001
SEED_TRAIN_SOURCE = 5000


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    for d in (lx, ly, lz, lt):
        if d < 2 or d % 2:
            raise ValueError(f"every lattice extent must be even and >= 2, got {dims}")
    return (lt, lz, ly, lx)


def volume(dims) -> int:
    lx, ly, lz, lt = dims
    return int(lx) * int(ly) * int(lz) * int(lt)


def complex_gaussian(g: np.random.Generator, shape) -> np.ndarray:
    """Complex normal with E|z|^2 = 1: (N(0,1) + i N(0,1)) / sqrt(2)."""
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def haar_su3(g: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices.

    QR of a complex Gaussian matrix, with the column phases fixed by the
    diagonal of R (Mezzadri's recipe for Haar U(3)), then divided by a cube
    root of the determinant so that det = 1.
    """
    z = complex_gaussian(g, (n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1] = -1j
_GELL_MANN[1][1, 0] = 1j
_GELL_MANN[2][0, 0] = 1
_GELL_MANN[2][1, 1] = -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2] = -1j
_GELL_MANN[4][2, 0] = 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2] = -1j
_GELL_MANN[6][2, 1] = 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def project_su3(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt of rows 0 and 1, third row = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def smooth_su3(g: np.random.Generator, n: int, eps: float = 0.3,
               chunk: int = 1 << 20) -> np.ndarray:
    """n matrices proj_SU3(exp(i*eps*H)), H = sum_a w_a lambda_a / 2, w_a ~ N(0,1)."""
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        w = g.standard_normal((hi - lo, 8))
        h = np.einsum("na,aij->nij", w, _GELL_MANN) * 0.5
        ev, vec = np.linalg.eigh(h)
        ph = np.exp(1j * eps * ev)
        u = np.einsum("nij,nj,nkj->nik", vec, ph, vec.conj())
        out[lo:hi] = project_su3(u)
    return out


def gauge_field(dims, kind: str, seed: int, eps: float = 0.3) -> np.ndarray:
    """Full-lattice gauge field U[t,z,y,x,mu,a,b] (complex128).

    kind: "unit" (free field), "haar" or "smooth".
    """
    shp = lattice_shape(dims)
    n = volume(dims) * 4
    if kind == "unit":
        u = np.broadcast_to(np.eye(3, dtype=np.complex128), (n, 3, 3)).copy()
    elif kind == "haar":
        u = haar_su3(rng(seed), n)
    elif kind == "smooth":
        u = smooth_su3(rng(seed), n, eps)
    else:
        raise ValueError(f"unknown gauge kind {kind!r}")
    return u.reshape(shp + (4, 3, 3))


def gauge_transform(dims, seed: int) -> np.ndarray:
    """Haar-random g(x) in SU(3) per site, shape (Lt,Lz,Ly,Lx,3,3)."""
    shp = lattice_shape(dims)
    return haar_su3(rng(seed), volume(dims)).reshape(shp + (3, 3))


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Full-lattice spinor with i.i.d. complex Gaussian components."""
    shp = lattice_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (nrhs,) + shp
    return complex_gaussian(rng(seed), shp)


def point_source(dims, spin: int, colour: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """delta_{x,site} delta_{s,spin} delta_{a,colour}; site given as (x0,x1,x2,x3)."""
    shp = lattice_shape(dims)
    psi = np.zeros(shp + (4, 3), dtype=np.complex128)
    x0, x1, x2, x3 = site
    psi[x3, x2, x1, x0, spin, colour] = 1.0
    return psi


def point_sources_12(dims) -> np.ndarray:
    """The 12 spin-colour point sources at the origin, RHS index r = 3*spin + colour."""
    return np.stack([point_source(dims, r // 3, r % 3) for r in range(12)])


def uneven_batch(seed: int = SEED_GAUGE + 3):
    """The eight lattices of the uneven batch and their hopping parameters.

    kappa_j ~ U[0.130, 0.136]; the returned list holds (dims, kappa, gauge
    seed, source seed) per solve.
    """
    lats = [(8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (16, 16, 16, 32),
            (16, 16, 16, 32), (20, 20, 20, 40), (24, 24, 24, 48), (24, 24, 24, 48)]
    g = rng(seed)
    kappas = g.uniform(0.130, 0.136, size=len(lats))
    return [(d, float(k), SEED_GAUGE + 30 + j, SEED_SOURCE + 30 + j)
            for j, (d, k) in enumerate(zip(lats, kappas))]
