// Flexible GMRES with deflated restarting (FGMRES-DR) on FP32 fields, with
// the residual recomputed in FP64 at every restart (section 7 of the paper:
// its SAP-FGMRES-DR keeps approximate eigenvectors in the Krylov subspace
// across restarts, after Morgan's GMRES-DR; section 5: iterative refinement
// at the restarts of the flexible solver).
//
// A cycle builds the flexible Arnoldi relation A Z_j = V_{j+1} Hbar_j with
// z_i = K v_i (K the preconditioner, which may change between calls) and
// classical Gram-Schmidt applied twice, solves min |c - Hbar y| by Givens
// rotations, and adds Z y to the FP64 solution.  At a restart the k
// harmonic Ritz vectors g_i of Hbar of smallest |theta| give the deflation
// directions Zd = Z G.  Their images A Zd are recomputed and orthonormalised
// (A Zd R^-1 = C, Zd <- Zd R^-1), so that A Zd = C holds to FP32 rounding
// whatever the FP64 residual turns out to be.  The next cycle then starts
// with V = [C, v], v the part of the FP64 residual orthogonal to C, and Hbar
// = [I_k 0; 0 0] in its first k columns.  In exact arithmetic this spans
// what Morgan's restart spans (span(A Zd) plus the residual), so it is the
// same method; it also lets the FP32 cycle start from a freshly computed
// FP64 residual (the paper's iterative refinement), which Morgan's form,
// carrying the old least-squares residual, would not.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "lq_internal.h"
#include "reduce.h"
#include "small_dense.h"

namespace lq {

namespace {

using cplx = std::complex<double>;
constexpr int KE = 4;  // entries per thread in the batched kernels

// Which entries of an FP32 field belong to sites: a field is one or two
// halves of per_half entries; in each half only the last 64-site block has
// padding, entries below lim are all live and in the last block the sites
// below rem (the chunked FP32 layout: site_in_block32).
struct Live {
  int64_t per_half, lim;
  int rem;
};
__device__ __forceinline__ bool kr_live(int64_t i, const Live& L) {
  const int64_t k = i < L.per_half ? i : i - L.per_half;
  return k < L.lim || site_in_block32(k) < L.rem;
}

// part[(j G + b) 2 + c]: workgroup b's partial of <V_j, x>
__global__ __launch_bounds__(256) void kr_mdot_kernel(const float2* const* __restrict__ V, int nv,
                                                      const float2* __restrict__ x, int64_t n,
                                                      Live L,
                                                      double* __restrict__ part) {
  float2 xv[KE];
  int64_t idx[KE];
  bool live[KE];
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    idx[e] = ((int64_t)blockIdx.x * KE + e) * 256 + threadIdx.x;
    live[e] = idx[e] < n && kr_live(idx[e], L);
    xv[e] = live[e] ? x[idx[e]] : make_float2(0.f, 0.f);
  }
  for (int j = 0; j < nv; ++j) {
    const float2* v = V[j];
    double a[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < KE; ++e)
      if (live[e]) {
        const float2 u = v[idx[e]];
        a[0] += (double)u.x * xv[e].x + (double)u.y * xv[e].y;
        a[1] += (double)u.x * xv[e].y - (double)u.y * xv[e].x;
      }
    block_partial_at<2>(a, part, (int64_t)j * gridDim.x + blockIdx.x);
  }
}

__global__ __launch_bounds__(256) void kr_mdot_fin_kernel(const double* __restrict__ part, int G,
                                                          double* __restrict__ res) {
  __shared__ double sh[2][16];
  const int j = blockIdx.x;
  double a[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < G; b += blockDim.x) {
    a[0] += part[((int64_t)j * G + b) * 2];
    a[1] += part[((int64_t)j * G + b) * 2 + 1];
  }
  block_sum<2>(a, sh);
  if (threadIdx.x == 0) {
    res[2 * j] = a[0];
    res[2 * j + 1] = a[1];
  }
}

// y -= sum_j c_j V_j, over the live entries
__global__ __launch_bounds__(256) void kr_maxpy_kernel(float2* __restrict__ y,
                                                       const float2* const* __restrict__ V,
                                                       const float2* __restrict__ c, int nv,
                                                       int64_t n, Live L) {
  float2 yv[KE];
  int64_t idx[KE];
  bool live[KE];
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    idx[e] = ((int64_t)blockIdx.x * KE + e) * 256 + threadIdx.x;
    live[e] = idx[e] < n && kr_live(idx[e], L);
    yv[e] = live[e] ? y[idx[e]] : make_float2(0.f, 0.f);
  }
  for (int j = 0; j < nv; ++j) {
    const float2 cj = c[j];
    const float2* v = V[j];
#pragma unroll
    for (int e = 0; e < KE; ++e)
      if (live[e]) {
        const float2 u = v[idx[e]];
        yv[e].x -= cj.x * u.x - cj.y * u.y;
        yv[e].y -= cj.x * u.y + cj.y * u.x;
      }
  }
#pragma unroll
  for (int e = 0; e < KE; ++e)
    if (live[e]) y[idx[e]] = yv[e];
}

// out_a = sum_i coef[i * nout + a] in_i for a < nout <= NMAX (out never
// aliases in); every input is read once, the NMAX sums stay in registers
constexpr int KR_MAXOUT = 32;
template <int NMAX>
__global__ __launch_bounds__(256) void kr_lincomb_kernel(float2* const* __restrict__ out, int nout,
                                                         const float2* const* __restrict__ in,
                                                         int nin, const float2* __restrict__ coef,
                                                         int64_t n, Live L) {
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i0 >= n || !kr_live(i0, L)) return;
  float2 acc[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) acc[a] = make_float2(0.f, 0.f);
  for (int i = 0; i < nin; ++i) {
    const float2 u = in[i][i0];
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
      if (a < nout) {
        const float2 c = coef[i * nout + a];
        acc[a].x += c.x * u.x - c.y * u.y;
        acc[a].y += c.x * u.y + c.y * u.x;
      }
  }
#pragma unroll
  for (int a = 0; a < NMAX; ++a)
    if (a < nout) out[a][i0] = acc[a];
}

// y = a x (complex a), live entries
__global__ void kr_scale_kernel(float2* __restrict__ y, float ar, float ai,
                                const float2* __restrict__ x, int64_t n, Live L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !kr_live(i, L)) return;
  const float2 u = x[i];
  y[i] = make_float2(ar * u.x - ai * u.y, ar * u.y + ai * u.x);
}

// out = s * in rounded to FP32 (s = 1 / |in| keeps any FP64 magnitude in range)
// (i counts FP32 entries; the FP64 entry of the same site and component is
// flat32_to_64(i))
__global__ void kr_to32_kernel(float2* __restrict__ out, const double2* __restrict__ in, double s,
                               int64_t n, Live L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !kr_live(i, L)) return;
  const double2 v = in[flat32_to_64(i)];
  out[i] = make_float2((float)(s * v.x), (float)(s * v.y));
}

// y += s * x (FP64 += FP32)
__global__ void kr_add64_kernel(double2* __restrict__ y, const float2* __restrict__ x, double s,
                                int64_t n, Live L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !kr_live(i, L)) return;
  const int64_t i64 = flat32_to_64(i);
  double2 v = y[i64];
  v.x += s * (double)x[i].x;
  v.y += s * (double)x[i].y;
  y[i64] = v;
}

void* kalloc(size_t bytes) {
  void* p = nullptr;
  LQ_HIP(hipMalloc(&p, bytes));
  return p;
}

}  // namespace

// Device work space of the deflated solver (lazily grown; freed with the context).
struct KrylovWork {
  int64_t n = 0;  // complex entries per field it was sized for
  std::vector<void*> V, Z, Zd;
  void* W = nullptr;   // the new Arnoldi vector before normalisation
  void* xc = nullptr;  // FP32 correction of a cycle
  void** vdev = nullptr;   // device arrays of field pointers
  void** zdev = nullptr;
  void** ddev = nullptr;
  double* part = nullptr;  // [nv][G][2] partials
  double* res = nullptr;   // [nv][2] dot products
  double* hres = nullptr;  // pinned host copy
  float2* coef = nullptr;  // coefficients (device)
  float2* hcoef = nullptr; // pinned host staging
  int cap_v = 0, cap_d = 0, cap_g = 0;
};

void free_krylov(lq_ctx* ctx) {
  KrylovWork* w = ctx->kwork;
  if (!w) return;
  for (auto* vec : {&w->V, &w->Z, &w->Zd})
    for (void* p : *vec) (void)hipFree(p);
  for (void* p : {w->W, w->xc, (void*)w->vdev, (void*)w->zdev, (void*)w->ddev, (void*)w->part,
                  (void*)w->res, (void*)w->coef})
    if (p) (void)hipFree(p);
  if (w->hres) (void)hipHostFree(w->hres);
  if (w->hcoef) (void)hipHostFree(w->hcoef);
  delete w;
  ctx->kwork = nullptr;
}

namespace {

struct Dr {
  lq_ctx* ctx;
  const KrylovSpace& S;
  KrylovWork* w;
  int G;  // workgroups of the batched kernels
  Live L;

  Dr(lq_ctx* c, const KrylovSpace& s, KrylovWork* kw)
      : ctx(c), S(s), w(kw), G(grid_for(s.n, 256 * KE)) {
    L.per_half = s.n / s.halves;
    const int64_t nblk = L.per_half / (12 * SB);
    L.lim = (nblk - 1) * 12 * SB;
    L.rem = (int)(s.vh - (nblk - 1) * SB);
  }

  // Device pointer arrays: vdev = V, zdev = Z, ddev = Zd then, at the
  // fixed slots KR_MAXOUT and KR_MAXOUT + 1, W and xc.  (Synchronous
  // copies: the host arrays change between calls.)
  void sync_ptrs() {
    LQ_HIP(hipStreamSynchronize(ctx->cur));  // no launch may still read the old arrays
    std::vector<void*> d(KR_MAXOUT + 2, nullptr);
    for (size_t i = 0; i < w->Zd.size(); ++i) d[i] = w->Zd[i];
    d[KR_MAXOUT] = w->W;
    d[KR_MAXOUT + 1] = w->xc;
    LQ_HIP(hipMemcpyAsync(w->vdev, w->V.data(), sizeof(void*) * w->V.size(),
                          hipMemcpyHostToDevice, ctx->cur));
    LQ_HIP(hipMemcpyAsync(w->zdev, w->Z.data(), sizeof(void*) * w->Z.size(),
                          hipMemcpyHostToDevice, ctx->cur));
    LQ_HIP(hipMemcpyAsync(w->ddev, d.data(), sizeof(void*) * d.size(), hipMemcpyHostToDevice,
                          ctx->cur));
    LQ_HIP(hipStreamSynchronize(ctx->cur));
  }
  // <P_j, x> for the nv fields at pointer array pdev (host results in w->hres)
  void mdot(void* const* pdev, int nv, const void* x) {
    hipLaunchKernelGGL(kr_mdot_kernel, dim3(G), dim3(256), 0, ctx->cur,
                       reinterpret_cast<const float2* const*>(pdev), nv,
                       reinterpret_cast<const float2*>(x), S.n, L, w->part);
    hipLaunchKernelGGL(kr_mdot_fin_kernel, dim3(nv), dim3(256), 0, ctx->cur, w->part, G, w->res);
    LQ_HIP(hipGetLastError());
    LQ_HIP(hipMemcpyAsync(w->hres, w->res, sizeof(double) * 2 * nv, hipMemcpyDeviceToHost,
                          ctx->cur));
    LQ_HIP(hipStreamSynchronize(ctx->cur));
    ctx->bytes += (double)S.n * 8 * (nv + 1);
  }
  double norm2_W() {  // |W|^2
    mdot(w->ddev + KR_MAXOUT, 1, w->W);
    return w->hres[0];
  }
  void upload_coef(const std::vector<cplx>& c) {
    LQ_CHECK(c.size() <= (size_t)129 * KR_MAXOUT, LQ_EINVAL, "FGMRES-DR: too many coefficients");
    LQ_HIP(hipStreamSynchronize(ctx->cur));  // the staging buffer's last copy has run
    for (size_t i = 0; i < c.size(); ++i)
      w->hcoef[i] = make_float2((float)c[i].real(), (float)c[i].imag());
    LQ_HIP(hipMemcpyAsync(w->coef, w->hcoef, sizeof(float2) * c.size(), hipMemcpyHostToDevice,
                          ctx->cur));
  }
  // y -= sum_j c_j P_j with the coefficients already on the device
  void maxpy(void* y, void* const* pdev, int nv) {
    hipLaunchKernelGGL(kr_maxpy_kernel, dim3(G), dim3(256), 0, ctx->cur,
                       reinterpret_cast<float2*>(y), reinterpret_cast<const float2* const*>(pdev),
                       w->coef, nv, S.n, L);
    LQ_HIP(hipGetLastError());
    ctx->bytes += (double)S.n * 8 * (nv + 2);
  }
  void scale(void* y, cplx a, const void* x) {
    hipLaunchKernelGGL(kr_scale_kernel, dim3(grid_for(S.n, 256)), dim3(256), 0, ctx->cur,
                       reinterpret_cast<float2*>(y), (float)a.real(), (float)a.imag(),
                       reinterpret_cast<const float2*>(x), S.n, L);
    LQ_HIP(hipGetLastError());
    ctx->bytes += (double)S.n * 16;
  }
  // Orthogonalise x against the nv orthonormal fields at vdev (classical
  // Gram-Schmidt, twice); the same combination is taken off z (at zdev) when
  // z is given.  Returns the summed coefficients.
  std::vector<cplx> orthogonalise(void* x, int nv, void* z) {
    std::vector<cplx> h(nv, 0.0);
    if (nv == 0) return h;
    for (int pass = 0; pass < 2; ++pass) {
      mdot(w->vdev, nv, x);
      std::vector<cplx> c(nv);
      for (int i = 0; i < nv; ++i) {
        c[i] = cplx(w->hres[2 * i], w->hres[2 * i + 1]);
        h[i] += c[i];
      }
      upload_coef(c);
      maxpy(x, w->vdev, nv);
      if (z) maxpy(z, w->zdev, nv);
    }
    return h;
  }
};

}  // namespace

bool fgmres_dr(lq_ctx* ctx, const KrylovSpace& S, int m, int k, double target, int maxiter,
               SolveTally& ss, bool& breakdown) {
  LQ_CHECK(m >= 2 && m <= 128, LQ_EINVAL, "FGMRES-DR: Krylov dimension m must be 2..128");
  LQ_CHECK(k >= 0 && k < m && k <= KR_MAXOUT, LQ_EINVAL,
           "FGMRES-DR: deflated vectors k must be 0..min(m-1, 32)");
  if (!ctx->kwork) ctx->kwork = new KrylovWork();
  KrylovWork* w = ctx->kwork;
  const size_t fb = (size_t)S.n * sizeof(float2);
  if (w->n != S.n) {  // another field shape: start over
    free_krylov(ctx);
    ctx->kwork = w = new KrylovWork();
    w->n = S.n;
  }
  while ((int)w->V.size() < m + 1) w->V.push_back(kalloc(fb));
  while ((int)w->Z.size() < m) w->Z.push_back(kalloc(fb));
  while ((int)w->Zd.size() < k) w->Zd.push_back(kalloc(fb));
  if (!w->W) w->W = kalloc(fb);
  if (!w->xc) w->xc = kalloc(fb);
  const int G = grid_for(S.n, 256 * KE);
  if (w->cap_v < m + 1 || w->cap_d < k + 1 || w->cap_g < G) {
    for (void* p : {(void*)w->vdev, (void*)w->zdev, (void*)w->ddev, (void*)w->part,
                    (void*)w->res, (void*)w->coef})
      if (p) (void)hipFree(p);
    if (w->hres) (void)hipHostFree(w->hres);
    if (w->hcoef) (void)hipHostFree(w->hcoef);
    const int nv = 129;
    w->vdev = reinterpret_cast<void**>(kalloc(sizeof(void*) * nv));
    w->zdev = reinterpret_cast<void**>(kalloc(sizeof(void*) * nv));
    w->ddev = reinterpret_cast<void**>(kalloc(sizeof(void*) * (KR_MAXOUT + 2)));
    w->part = reinterpret_cast<double*>(kalloc(sizeof(double) * 2 * (size_t)G * nv));
    w->res = reinterpret_cast<double*>(kalloc(sizeof(double) * 2 * nv));
    w->coef = reinterpret_cast<float2*>(kalloc(sizeof(float2) * nv * KR_MAXOUT));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->hres), sizeof(double) * 2 * nv));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->hcoef), sizeof(float2) * nv * KR_MAXOUT));
    w->cap_v = nv - 1;
    w->cap_d = KR_MAXOUT;
    w->cap_g = G;
  }
  Dr dr(ctx, S, w);
  dr.sync_ptrs();
  std::vector<void*>& V = w->V;
  std::vector<void*>& Z = w->Z;
  int kd = 0;  // deflation vectors waiting in Zd
  double best = INFINITY;
  int stalls = 0;
  for (;;) {
    // ---- restart: FP64 residual, stopping and stall tests
    const double beta = std::sqrt(S.residual64());
    if (!std::isfinite(beta)) {
      breakdown = true;
      return false;
    }
    if (beta <= target) return true;
    if (ss.iterations >= maxiter) return false;
    if (beta < 0.5 * best) {
      best = beta;
      stalls = 0;
    } else if (++stalls >= 3) {
      breakdown = true;
      return false;
    }
    ss.reliable += 1;
    // ---- the deflation directions: A Zd orthonormalised into V[0..kd)
    std::vector<cplx> H((size_t)(m + 1) * m, 0.0), Hraw((size_t)(m + 1) * m, 0.0);
    std::vector<cplx> g(m + 1, 0.0), sn(m, 0.0);
    std::vector<double> cs(m, 1.0);
    int j0 = 0;
    for (int a = 0; a < kd; ++a) {
      std::swap(Z[a], w->Zd[a]);
      dr.sync_ptrs();
      S.op(w->W, Z[a]);
      const double an = std::sqrt(dr.norm2_W());
      (void)dr.orthogonalise(w->W, a, Z[a]);
      const double rn = std::sqrt(dr.norm2_W());
      if (!(rn > 1e-4 * an) || !std::isfinite(rn)) break;  // (nearly) dependent: stop here
      dr.scale(V[a], 1.0 / rn, w->W);
      dr.scale(Z[a], 1.0 / rn, Z[a]);
      H[(size_t)a * m + a] = Hraw[(size_t)a * m + a] = 1.0;
      j0 = a + 1;
    }
    dr.sync_ptrs();
    // ---- the FP64 residual, normalised, minus its part in C
    hipLaunchKernelGGL(kr_to32_kernel, dim3(grid_for(S.n, 256)), dim3(256), 0, ctx->cur,
                       reinterpret_cast<float2*>(w->W), reinterpret_cast<const double2*>(S.r64),
                       1.0 / beta, S.n, dr.L);
    LQ_HIP(hipGetLastError());
    const std::vector<cplx> c = dr.orthogonalise(w->W, j0, nullptr);
    for (int a = 0; a < j0; ++a) g[a] = c[a];
    const double eta = std::sqrt(dr.norm2_W());
    if (!std::isfinite(eta)) {
      breakdown = true;
      return false;
    }
    g[j0] = eta;
    if (eta > 0.0) dr.scale(V[j0], 1.0 / eta, w->W);
    // an FP32 cycle reduces its residual by about 1e-5 reliably; the last
    // stops at what the FP64 residual still needs (with a margin of 2)
    const double cycle_tol = std::max(1e-5, 0.5 * target / beta);
    int jend = j0;
    if (eta > cycle_tol) {
      for (int j = j0; j < m && ss.iterations < maxiter; ++j) {
        S.precond(Z[j], V[j]);
        S.op(w->W, Z[j]);
        ss.iterations += 1;
        const std::vector<cplx> h = dr.orthogonalise(w->W, j + 1, nullptr);
        const double hn = std::sqrt(dr.norm2_W());
        if (!std::isfinite(hn)) {
          breakdown = true;
          return false;
        }
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = Hraw[(size_t)i * m + j] = h[i];
        H[(size_t)(j + 1) * m + j] = Hraw[(size_t)(j + 1) * m + j] = hn;
        if (hn > 0.0) dr.scale(V[j + 1], 1.0 / hn, w->W);
        for (int i = 0; i < j; ++i) {  // earlier rotations, then the one clearing H[j+1][j]
          const cplx a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
          H[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * b;
        }
        double cr;
        cplx sr;
        dense::givens(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j], cr, sr);
        cs[j] = cr;
        sn[j] = sr;
        const cplx a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
        H[(size_t)j * m + j] = cr * a + sr * b;
        H[(size_t)(j + 1) * m + j] = 0.0;
        g[j + 1] = -std::conj(sr) * g[j];
        g[j] = cr * g[j];
        jend = j + 1;
        if (std::abs(g[j + 1]) <= cycle_tol || hn == 0.0) break;
      }
    }
    // ---- y = R^-1 g, x += beta Z y
    std::vector<cplx> y(jend);
    for (int i = jend - 1; i >= 0; --i) {
      cplx t = g[i];
      for (int j = i + 1; j < jend; ++j) t -= H[(size_t)i * m + j] * y[j];
      y[i] = t / H[(size_t)i * m + i];
      if (!std::isfinite(y[i].real()) || !std::isfinite(y[i].imag())) {
        breakdown = true;
        return false;
      }
    }
    if (jend > 0) {
      dr.upload_coef(y);
      hipLaunchKernelGGL(kr_lincomb_kernel<1>, dim3(grid_for(S.n, 256)), dim3(256), 0, ctx->cur,
                         reinterpret_cast<float2* const*>(w->ddev + KR_MAXOUT + 1), 1,
                         reinterpret_cast<const float2* const*>(w->zdev), jend, w->coef, S.n, dr.L);
      hipLaunchKernelGGL(kr_add64_kernel, dim3(grid_for(S.n, 256)), dim3(256), 0, ctx->cur,
                         reinterpret_cast<double2*>(S.x64),
                         reinterpret_cast<const float2*>(w->xc), beta, S.n, dr.L);
      LQ_HIP(hipGetLastError());
      ctx->bytes += (double)S.n * (8.0 * (jend + 1) + 32.0);
    }
    // ---- deflation directions for the next cycle: Zd = Z G (harmonic Ritz)
    kd = 0;
    if (k > 0 && jend > k) {
      std::vector<cplx> gv, theta;
      if (dense::harmonic_ritz(jend, Hraw, m, k, gv, theta)) {
        std::vector<cplx> coef((size_t)jend * k);
        for (int i = 0; i < jend; ++i)
          for (int a = 0; a < k; ++a) coef[(size_t)i * k + a] = gv[(size_t)i * k + a];
        dr.upload_coef(coef);
        auto lc = [&](auto kern) {
          hipLaunchKernelGGL(kern, dim3(grid_for(S.n, 256)), dim3(256), 0, ctx->cur,
                             reinterpret_cast<float2* const*>(w->ddev), k,
                             reinterpret_cast<const float2* const*>(w->zdev), jend, w->coef, S.n,
                             dr.L);
        };
        if (k <= 8)
          lc(kr_lincomb_kernel<8>);
        else if (k <= 16)
          lc(kr_lincomb_kernel<16>);
        else
          lc(kr_lincomb_kernel<32>);
        LQ_HIP(hipGetLastError());
        ctx->bytes += (double)S.n * 8.0 * (jend + k);
        kd = k;
      }
    }
  }
}

}  // namespace lq
