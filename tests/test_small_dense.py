"""Host check of the small dense routines the deflated FGMRES restarts use
(csrc/small_dense.h, built with g++): the Hessenberg eigen-solver against
NumPy's eigenvalues, and the harmonic Ritz values against the oracle's
(oracle.solvers.harmonic_ritz, built on NumPy's eig), each with its own
residual check."""
import os
import subprocess

import numpy as np
import pytest

from oracle import solvers

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("dense") / "small_dense_check")
    src = os.path.join(HERE, "host", "small_dense_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, src], check=True)
    return exe


def run(exe, header, mat):
    text = header + "\n" + "\n".join(f"{v.real:.17g} {v.imag:.17g}" for v in mat.reshape(-1))
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.split("\n")
    resid = float(lines[0].split()[1])
    vals = np.array([complex(float(a), float(b)) for a, b in
                     (ln.split() for ln in lines[1:] if ln.strip())])
    return resid, vals


def match(a, b):
    """Largest distance from an entry of a to its nearest entry of b."""
    return max(np.min(np.abs(b - x)) for x in a)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (30, 3), (70, 4)])
def test_hessenberg_eigenpairs(checker, n, seed):
    rng = np.random.default_rng(seed)
    a = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
    resid, w = run(checker, f"eig {n}", a)
    assert resid <= 1e-11
    ev = np.linalg.eigvals(a)
    assert match(w, ev) <= 1e-9 * max(1.0, np.abs(ev).max())
    assert match(ev, w) <= 1e-9 * max(1.0, np.abs(ev).max())


def test_hessenberg_with_repeated_and_zero_subdiagonals(checker):
    """A block-triangular case (zero subdiagonal entries) and a diagonal
    with repeated eigenvalues."""
    a = np.diag([2.0 + 0j, 2.0, -1.0, 0.5j, 0.5j]) + np.diag([1.0, 0, 0.3, 0], 1)
    resid, w = run(checker, "eig 5", a)
    assert resid <= 1e-12
    assert match(w, np.diag(a)) <= 1e-12


@pytest.mark.parametrize("j,k,seed", [(12, 4, 5), (40, 10, 6), (70, 10, 7)])
def test_harmonic_ritz_against_oracle(checker, j, k, seed):
    rng = np.random.default_rng(seed)
    h = np.triu(rng.standard_normal((j + 1, j)) + 1j * rng.standard_normal((j + 1, j)), -1)
    resid, th = run(checker, f"hritz {j} {k}", h)
    assert resid <= 1e-10
    ref, _ = solvers.harmonic_ritz(h, k)
    assert match(th, ref) <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("n,seed", [(1, 20), (3, 21), (12, 22), (16, 23)])
def test_hermitian_eigen(checker, n, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = z @ z.conj().T
    resid, w = run(checker, f"herm {n}", a)
    assert resid <= 1e-12
    assert np.allclose(np.sort(w.real), np.linalg.eigvalsh(a), rtol=1e-11, atol=1e-12 * n)


def test_hermitian_eigen_rank_deficient(checker):
    """A Gram matrix of dependent columns: the zero eigenvalues come out at
    rounding level, the others exact."""
    rng = np.random.default_rng(24)
    b = rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))
    cols = np.concatenate([b, b[:, :1] * 2j, b[:, 1:2] + b[:, 2:3]], axis=1)
    a = cols.conj().T @ cols
    resid, w = run(checker, "herm 5", a)
    assert resid <= 1e-12
    ref = np.linalg.eigvalsh(a)
    assert np.allclose(np.sort(w.real)[2:], ref[2:], rtol=1e-11)
    assert np.all(np.abs(np.sort(w.real)[:2]) <= 1e-12 * ref[-1])
