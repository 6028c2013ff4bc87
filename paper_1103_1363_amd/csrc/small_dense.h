// Small dense complex linear algebra on the host, for the restarts of the
// deflated flexible GMRES: a linear solve, the eigenpairs of an upper
// Hessenberg matrix, and the harmonic Ritz vectors of an Arnoldi matrix.
// Sizes are the Krylov dimension (at most a few hundred), so plain loops.
//
// Plain C++ (no device code) so that the host tests can build it with g++.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace lq {
namespace dense {

using cplx = std::complex<double>;

// Solve A x = b (A n x n row-major, overwritten by its LU factors) by
// Gaussian elimination with partial pivoting.  Returns false if A is
// singular to working precision.
inline bool solve(int n, std::vector<cplx>& a, std::vector<cplx>& b) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(a[(size_t)r * n + c]) > std::abs(a[(size_t)p * n + c])) p = r;
    if (std::abs(a[(size_t)p * n + c]) == 0.0) return false;
    if (p != c) {
      for (int k = 0; k < n; ++k) std::swap(a[(size_t)p * n + k], a[(size_t)c * n + k]);
      std::swap(b[p], b[c]);
    }
    const cplx d = a[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      const cplx f = a[(size_t)r * n + c] / d;
      if (f == cplx(0.0)) continue;
      for (int k = c; k < n; ++k) a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    cplx t = b[r];
    for (int k = r + 1; k < n; ++k) t -= a[(size_t)r * n + k] * b[k];
    b[r] = t / a[(size_t)r * n + r];
  }
  return true;
}

// Rotation [c, s; -conj(s), c] (c real) that maps (x, y) to (r, 0).
inline void givens(cplx x, cplx y, double& c, cplx& s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = std::conj(y) / ay;
    return;
  }
  const double nrm = std::hypot(ax, ay);
  c = ax / nrm;
  s = (x / ax) * std::conj(y) / nrm;
}

// Eigenvalues w[n] and unit eigenvectors (columns of x, n x n row-major) of
// the complex upper Hessenberg matrix h (n x n row-major, destroyed), by the
// single-shift QR algorithm with Wilkinson shifts and Givens rotations to
// the Schur form T = Q^dagger h Q, then back substitution on T.  Returns
// false if the iteration does not converge (30 n sweeps).
inline bool hessenberg_eig(int n, std::vector<cplx>& h, std::vector<cplx>& w,
                           std::vector<cplx>& x) {
  auto H = [&](int r, int c) -> cplx& { return h[(size_t)r * n + c]; };
  std::vector<cplx> q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      const double s = std::abs(H(l - 1, l - 1)) + std::abs(H(l, l));
      if (std::abs(H(l, l - 1)) <= eps * (s > 0.0 ? s : 1.0)) break;
      --l;
    }
    if (l > 0) H(l, l - 1) = 0.0;
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 30 * n) return false;
    ++iter;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 nearer to its corner
    const cplx a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    const cplx tr = a + d, det = a * d - b * c;
    const cplx disc = std::sqrt(tr * tr / 4.0 - det);
    const cplx m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
    cplx mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    if (iter % 11 == 10) mu = d + std::abs(c);  // exceptional shift against cycling
    // implicit QR step on rows/columns l..hi: the first rotation from the
    // shifted first column, the rest chase the bulge down the subdiagonal
    for (int k = l; k < hi; ++k) {
      const cplx xk = k == l ? H(l, l) - mu : H(k, k - 1);
      const cplx yk = k == l ? H(l + 1, l) : H(k + 1, k - 1);
      double cr;
      cplx sn;
      givens(xk, yk, cr, sn);
      for (int col = (k == l ? l : k - 1); col < n; ++col) {
        const cplx u = H(k, col), v = H(k + 1, col);
        H(k, col) = cr * u + sn * v;
        H(k + 1, col) = -std::conj(sn) * u + cr * v;
      }
      if (k > l) H(k + 1, k - 1) = 0.0;
      const int rmax = std::min(k + 2, hi);
      for (int row = 0; row <= rmax; ++row) {
        const cplx u = H(row, k), v = H(row, k + 1);
        H(row, k) = cr * u + std::conj(sn) * v;
        H(row, k + 1) = -sn * u + cr * v;
      }
      for (int row = 0; row < n; ++row) {
        const cplx u = q[(size_t)row * n + k], v = q[(size_t)row * n + k + 1];
        q[(size_t)row * n + k] = cr * u + std::conj(sn) * v;
        q[(size_t)row * n + k + 1] = -sn * u + cr * v;
      }
    }
  }
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) w[i] = H(i, i);
  // eigenvectors of the triangular T, then x = Q y
  double tnorm = 0.0;
  for (int r = 0; r < n; ++r)
    for (int c2 = r; c2 < n; ++c2) tnorm = std::max(tnorm, std::abs(H(r, c2)));
  const double small = eps * (tnorm > 0.0 ? tnorm : 1.0);
  x.assign((size_t)n * n, 0.0);
  std::vector<cplx> y(n);
  for (int i = 0; i < n; ++i) {
    std::fill(y.begin(), y.end(), cplx(0.0));
    y[i] = 1.0;
    for (int j = i - 1; j >= 0; --j) {
      cplx t = 0.0;
      for (int k = j + 1; k <= i; ++k) t += H(j, k) * y[k];
      cplx den = H(j, j) - w[i];
      if (std::abs(den) < small) den = small;
      y[j] = -t / den;
    }
    double nrm = 0.0;
    for (int r = 0; r < n; ++r) {
      cplx t = 0.0;
      for (int k = 0; k <= i; ++k) t += q[(size_t)r * n + k] * y[k];
      x[(size_t)r * n + i] = t;
      nrm += std::norm(t);
    }
    nrm = std::sqrt(nrm);
    for (int r = 0; r < n; ++r) x[(size_t)r * n + i] /= nrm;
  }
  return true;
}

// Harmonic Ritz vectors of the (j+1) x j upper Hessenberg Arnoldi matrix
// hbar (row-major, row stride ld >= j): the eigenpairs of
// H_j + |h_{j+1,j}|^2 f e_j^dagger with H_j^dagger f = e_j, whose
// eigenvalues theta satisfy hbar^dagger (hbar g - theta [g; 0]) = 0.
// Returns the k (<= j) eigenvectors of smallest |theta| as the columns of
// g (j x k row-major) and their theta; false on a singular H_j or no QR
// convergence.
inline bool harmonic_ritz(int j, const std::vector<cplx>& hbar, int ld, int k,
                          std::vector<cplx>& g, std::vector<cplx>& theta) {
  std::vector<cplx> hm((size_t)j * j), a((size_t)j * j), f(j, 0.0);
  for (int r = 0; r < j; ++r)
    for (int c = 0; c < j; ++c) {
      hm[(size_t)r * j + c] = hbar[(size_t)r * ld + c];
      a[(size_t)r * j + c] = std::conj(hbar[(size_t)c * ld + r]);  // H_j^dagger
    }
  f[j - 1] = 1.0;
  if (!solve(j, a, f)) return false;
  const double h2 = std::norm(hbar[(size_t)j * ld + (j - 1)]);
  for (int r = 0; r < j; ++r) hm[(size_t)r * j + (j - 1)] += h2 * f[r];
  std::vector<cplx> w, x;
  if (!hessenberg_eig(j, hm, w, x)) return false;
  std::vector<int> order(j);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int p, int q2) { return std::abs(w[p]) < std::abs(w[q2]); });
  g.assign((size_t)j * k, 0.0);
  theta.assign(k, 0.0);
  for (int i = 0; i < k; ++i) {
    theta[i] = w[order[i]];
    for (int r = 0; r < j; ++r) g[(size_t)r * k + i] = x[(size_t)r * j + order[i]];
  }
  return true;
}

// Eigenvalues w[n] (ascending) and orthonormal eigenvectors (columns of v,
// n x n row-major) of the complex Hermitian matrix a (n x n row-major,
// destroyed) by cyclic Jacobi rotations: each pair (p, q) is made real by a
// phase and then cleared by the real Jacobi rotation of that 2 x 2 block.
inline void hermitian_eig(int n, std::vector<cplx>& a, std::vector<double>& w,
                          std::vector<cplx>& v) {
  auto A = [&](int r, int c) -> cplx& { return a[(size_t)r * n + c]; };
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  double norm = 0.0;
  for (const cplx& z : a) norm += std::norm(z);
  norm = std::sqrt(norm);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(A(p, q));
    if (std::sqrt(off) <= 1e-15 * (norm > 0.0 ? norm : 1.0)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = std::abs(A(p, q));
        if (apq == 0.0) continue;
        const cplx ph = A(p, q) / apq;  // a_pq = |a_pq| ph
        const double app = A(p, p).real(), aqq = A(q, q).real();
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        // G = [[c, sn ph], [-sn conj(ph), c]] on columns p, q: A <- G^+ A G
        const cplx gpq = sn * ph, gqp = -sn * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // columns
          const cplx akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp + gqp * akq;
          A(k, q) = gpq * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows (conjugate transpose of G)
          const cplx apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk + std::conj(gqp) * aqk;
          A(q, k) = std::conj(gpq) * apk + c * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const cplx vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp + gqp * vkq;
          v[(size_t)k * n + q] = gpq * vkp + c * vkq;
        }
      }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return A(x, x).real() < A(y, y).real(); });
  std::vector<cplx> vs((size_t)n * n);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    w[i] = A(order[i], order[i]).real();
    for (int r = 0; r < n; ++r) vs[(size_t)r * n + i] = v[(size_t)r * n + order[i]];
  }
  v.swap(vs);
}

}  // namespace dense
}  // namespace lq
