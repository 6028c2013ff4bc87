// Host check of the small dense routines (paper_1103_1363_amd/csrc/small_dense.h).
// Reads from stdin:
//   eig n  (n*n complex entries "re im", row-major, upper Hessenberg)
//     -> prints the eigenvalues and max_i |A x_i - w_i x_i| / max|A|
//   herm n  (n*n complex entries, Hermitian)
//     -> the ascending eigenvalues, and the largest of the eigen-residual
//        and the loss of orthonormality of the eigenvectors
//   hritz j k  ((j+1)*j complex entries, row-major)
//     -> prints the k harmonic Ritz values and the largest relative
//        Petrov-Galerkin residual |hbar^+ (hbar g - theta [g; 0])|
#include <cstdio>
#include <cstring>

#include "../../paper_1103_1363_amd/csrc/small_dense.h"

using lq::dense::cplx;

static std::vector<cplx> read_mat(int rows, int cols) {
  std::vector<cplx> a((size_t)rows * cols);
  for (auto& v : a) {
    double re = 0, im = 0;
    if (std::scanf("%lf %lf", &re, &im) != 2) std::exit(3);
    v = cplx(re, im);
  }
  return a;
}

int main() {
  char mode[16];
  if (std::scanf("%15s", mode) != 1) return 2;
  if (!std::strcmp(mode, "eig")) {
    int n;
    if (std::scanf("%d", &n) != 1) return 2;
    std::vector<cplx> a = read_mat(n, n), h = a, w, x;
    if (!lq::dense::hessenberg_eig(n, h, w, x)) {
      std::printf("noconv\n");
      return 1;
    }
    double amax = 0.0, worst = 0.0;
    for (auto& v : a) amax = std::max(amax, std::abs(v));
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < n; ++r) {
        cplx t = -w[i] * x[(size_t)r * n + i];
        for (int c = 0; c < n; ++c) t += a[(size_t)r * n + c] * x[(size_t)c * n + i];
        worst = std::max(worst, std::abs(t) / amax);
      }
    std::printf("resid %.3e\n", worst);
    for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", w[i].real(), w[i].imag());
    return 0;
  }
  if (!std::strcmp(mode, "hritz")) {
    int j, k;
    if (std::scanf("%d %d", &j, &k) != 2) return 2;
    std::vector<cplx> hb = read_mat(j + 1, j), g, th;
    if (!lq::dense::harmonic_ritz(j, hb, j, k, g, th)) {
      std::printf("fail\n");
      return 1;
    }
    double worst = 0.0, hn = 0.0;
    for (auto& v : hb) hn += std::norm(v);
    for (int i = 0; i < k; ++i) {
      std::vector<cplx> d(j + 1, 0.0);  // hbar g - theta [g; 0]
      for (int r = 0; r <= j; ++r) {
        cplx t = r < j ? -th[i] * g[(size_t)r * k + i] : cplx(0.0);
        for (int c = 0; c < j; ++c) t += hb[(size_t)r * j + c] * g[(size_t)c * k + i];
        d[r] = t;
      }
      for (int c = 0; c < j; ++c) {
        cplx t = 0.0;
        for (int r = 0; r <= j; ++r) t += std::conj(hb[(size_t)r * j + c]) * d[r];
        worst = std::max(worst, std::abs(t) / hn);
      }
    }
    std::printf("resid %.3e\n", worst);
    for (int i = 0; i < k; ++i) std::printf("%.17g %.17g\n", th[i].real(), th[i].imag());
    return 0;
  }
  if (!std::strcmp(mode, "herm")) {
    int n;
    if (std::scanf("%d", &n) != 1) return 2;
    std::vector<cplx> a = read_mat(n, n), h = a, v;
    std::vector<double> w;
    lq::dense::hermitian_eig(n, h, w, v);
    double amax = 0.0, worst = 0.0, orth = 0.0;
    for (auto& z : a) amax = std::max(amax, std::abs(z));
    for (int i = 0; i < n; ++i) {
      for (int r = 0; r < n; ++r) {
        cplx t = -w[i] * v[(size_t)r * n + i];
        for (int c = 0; c < n; ++c) t += a[(size_t)r * n + c] * v[(size_t)c * n + i];
        worst = std::max(worst, std::abs(t) / amax);
      }
      for (int j = 0; j < n; ++j) {
        cplx d = 0.0;
        for (int r = 0; r < n; ++r) d += std::conj(v[(size_t)r * n + i]) * v[(size_t)r * n + j];
        orth = std::max(orth, std::abs(d - (i == j ? 1.0 : 0.0)));
      }
    }
    std::printf("resid %.3e\n", std::max(worst, orth));
    for (int i = 0; i < n; ++i) std::printf("%.17g 0\n", w[i]);
    return 0;
  }
  return 2;
}
