// Clover term construction in FP64 on the GPU.
//
// Per site: the four mu->nu ordered plaquette leaves give Q_{mu nu}; the
// Hermitian traceless field strength is F = (Q - Q^+)/(8i) - tr/3.  In the
// chiral basis sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] is block diagonal:
//   sigma_{jk} = -eps_{jkl} diag(s_l, s_l)  (j,k,l spatial),
//   sigma_{k4} = diag(s_k, -s_k),
// so sum_{mu<nu} sigma F = diag(S_up, S_dn) with, for each chirality block,
//   S = [[Z, X - iY], [X + iY, -Z]]  (2 spins x 3 colours),
//   up:   X = F03 - F12,  Y = F13 + F02,  Z = F23 - F01,
//   down: X = -F03 - F12, Y = -F13 + F02, Z = -F23 - F01,
// (mu = 0..3 <-> x, y, z, t) and A = 1 - csw kappa diag(S_up, S_dn).
// Each 6x6 block is inverted by Gauss-Jordan elimination with partial
// pivoting in FP64.
#include "dslash_core.h"

namespace lq {

namespace {

using Cd = C<double>;

struct M3 {
  Cd m[9];
};

__device__ inline M3 mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cd acc = a.m[3 * i] * b.m[j];
      acc = acc + a.m[3 * i + 1] * b.m[3 + j];
      acc = acc + a.m[3 * i + 2] * b.m[6 + j];
      r.m[3 * i + j] = acc;
    }
  return r;
}
__device__ inline M3 dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[3 * i + j] = conj(a.m[3 * j + i]);
  return r;
}

// U_mu at full-lattice coordinates x + d (d an offset vector), periodic.
__device__ inline M3 link_at(const Geo& g, const double2* __restrict__ g64, const int x[4],
                             const int d[4], int mu) {
  int y[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int v = x[k] + d[k];
    v = v < 0 ? v + g.L[k] : (v >= g.L[k] ? v - g.L[k] : v);
    y[k] = v;
  }
  const int p = (y[0] + y[1] + y[2] + y[3]) & 1;
  M3 u;
  load_link<P64>(g64, g.nblk, p, mu, cb_index(g, y), u.m);
  return u;
}

// Hermitian traceless F_{mu nu}(x)
__device__ M3 field_strength(const Geo& g, const double2* __restrict__ g64, const int x[4], int mu,
                             int nu) {
  int d0[4] = {0, 0, 0, 0};
  int dpm[4], dpn[4], dmm[4], dmn[4], dmmpn[4], dpmmn[4], dmmmn[4];
  // explicit offsets (mu, nu) components
  for (int k = 0; k < 4; ++k) {
    dpm[k] = (k == mu) ? 1 : 0;
    dpn[k] = (k == nu) ? 1 : 0;
    dmm[k] = (k == mu) ? -1 : 0;
    dmn[k] = (k == nu) ? -1 : 0;
    dmmpn[k] = (k == mu) ? -1 : ((k == nu) ? 1 : 0);
    dpmmn[k] = (k == mu) ? 1 : ((k == nu) ? -1 : 0);
    dmmmn[k] = (k == mu || k == nu) ? -1 : 0;
  }
  const M3 um_x = link_at(g, g64, x, d0, mu);
  const M3 un_x = link_at(g, g64, x, d0, nu);
  // leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
  M3 q = mul(mul(um_x, link_at(g, g64, x, dpm, nu)), mul(dag(link_at(g, g64, x, dpn, mu)), dag(un_x)));
  // leaf 2: x -> x-nu -> x-nu+mu -> x+mu -> x
  M3 l2 = mul(mul(dag(link_at(g, g64, x, dmn, nu)), link_at(g, g64, x, dmn, mu)),
              mul(link_at(g, g64, x, dpmmn, nu), dag(um_x)));
  // leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
  M3 l3 = mul(mul(dag(link_at(g, g64, x, dmm, mu)), dag(link_at(g, g64, x, dmmmn, nu))),
              mul(link_at(g, g64, x, dmmmn, mu), link_at(g, g64, x, dmn, nu)));
  // leaf 4: x -> x+nu -> x+nu-mu -> x-mu -> x
  M3 l4 = mul(mul(un_x, dag(link_at(g, g64, x, dmmpn, mu))),
              mul(dag(link_at(g, g64, x, dmm, nu)), link_at(g, g64, x, dmm, mu)));
  for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l2.m[k] + l3.m[k] + l4.m[k];
  M3 f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Cd z = q.m[3 * i + j] - conj(q.m[3 * j + i]);  // (Q - Q^+)_{ij}
      f.m[3 * i + j] = Cd{z.im / 8.0, -z.re / 8.0};  // divided by 8i
    }
  const double tr = (f.m[0].re + f.m[4].re + f.m[8].re) / 3.0;
  f.m[0].re -= tr;
  f.m[4].re -= tr;
  f.m[8].re -= tr;
  return f;
}

// In-place inverse of a 6x6 complex matrix (Gauss-Jordan, partial pivoting).
__device__ void invert6(Cd a[36]) {
  Cd inv[36];
  for (int i = 0; i < 36; ++i) inv[i] = Cd{(i / 6 == i % 6) ? 1.0 : 0.0, 0.0};
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    double best = norm2(a[6 * col + col]);
    for (int r = col + 1; r < 6; ++r) {
      double v = norm2(a[6 * r + col]);
      if (v > best) best = v, piv = r;
    }
    if (piv != col)
      for (int k = 0; k < 6; ++k) {
        Cd t = a[6 * col + k];
        a[6 * col + k] = a[6 * piv + k];
        a[6 * piv + k] = t;
        t = inv[6 * col + k];
        inv[6 * col + k] = inv[6 * piv + k];
        inv[6 * piv + k] = t;
      }
    const Cd d = a[6 * col + col];
    const double dn = 1.0 / norm2(d);
    const Cd di = Cd{d.re * dn, -d.im * dn};
    for (int k = 0; k < 6; ++k) {
      a[6 * col + k] = a[6 * col + k] * di;
      inv[6 * col + k] = inv[6 * col + k] * di;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const Cd f = a[6 * r + col];
      for (int k = 0; k < 6; ++k) {
        a[6 * r + k] = a[6 * r + k] - f * a[6 * col + k];
        inv[6 * r + k] = inv[6 * r + k] - f * inv[6 * col + k];
      }
    }
  }
  for (int i = 0; i < 36; ++i) a[i] = inv[i];
}

template <class S>
__device__ inline void store_block(S* dst, int64_t s, int b, const Cd m[36]);

template <>
__device__ inline void store_block<double2>(double2* dst, int64_t s, int b, const Cd m[36]) {
  for (int k = 0; k < 3; ++k)
    dst[clov_idx(s, 18 * b + k)] = make_double2(m[7 * (2 * k)].re, m[7 * (2 * k + 1)].re);
  for (int r = 0; r < 6; ++r)
    for (int c = r + 1; c < 6; ++c) {
      const Cd v = m[6 * r + c];
      dst[clov_idx(s, 18 * b + 3 + tri_idx(r, c))] = make_double2(v.re, v.im);
    }
}
template <>
__device__ inline void store_block<float2>(float2* dst, int64_t s, int b, const Cd m[36]) {
  for (int k = 0; k < 3; ++k)
    dst[clov32_idx(s, 18 * b + k)] = make_float2((float)m[7 * (2 * k)].re, (float)m[7 * (2 * k + 1)].re);
  for (int r = 0; r < 6; ++r)
    for (int c = r + 1; c < 6; ++c) {
      const Cd v = m[6 * r + c];
      dst[clov32_idx(s, 18 * b + 3 + tri_idx(r, c))] = make_float2((float)v.re, (float)v.im);
    }
}
template <>
__device__ inline void store_block<__half2>(__half2* dst, int64_t s, int b, const Cd m[36]) {
  for (int k = 0; k < 3; ++k)
    dst[clov16_idx(s, 18 * b + k)] =
        __floats2half2_rn((float)m[7 * (2 * k)].re, (float)m[7 * (2 * k + 1)].re);
  for (int r = 0; r < 6; ++r)
    for (int c = r + 1; c < 6; ++c) {
      const Cd v = m[6 * r + c];
      dst[clov16_idx(s, 18 * b + 3 + tri_idx(r, c))] = __floats2half2_rn((float)v.re, (float)v.im);
    }
}

struct CloverOut {
  double2* a64[2];
  double2* ai64[2];
  float2* a32_ee;
  float2* ai32_oo;
  __half2* a16_ee;
  __half2* ai16_oo;
};

__global__ __launch_bounds__(128) void build_clover_kernel(Geo g, const double2* __restrict__ g64,
                                                           double ck, CloverOut out, int64_t V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  int x[4];
  canonical_coords(g, i, x);
  const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  const int64_t s = cb_index(g, x);
  M3 f01, f02, f03, f12, f13, f23;
  if (ck != 0.0) {
    f01 = field_strength(g, g64, x, 0, 1);
    f02 = field_strength(g, g64, x, 0, 2);
    f03 = field_strength(g, g64, x, 0, 3);
    f12 = field_strength(g, g64, x, 1, 2);
    f13 = field_strength(g, g64, x, 1, 3);
    f23 = field_strength(g, g64, x, 2, 3);
  } else {
    for (int k = 0; k < 9; ++k) f01.m[k] = f02.m[k] = f03.m[k] = f12.m[k] = f13.m[k] = f23.m[k] = Cd{0, 0};
  }
  for (int b = 0; b < 2; ++b) {
    const double sg = b == 0 ? 1.0 : -1.0;
    Cd a[36];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int k = 3 * r + c;
        const Cd X = sg * f03.m[k] - f12.m[k];
        const Cd Y = sg * f13.m[k] + f02.m[k];
        const Cd Z = sg * f23.m[k] - f01.m[k];
        const Cd one = Cd{r == c ? 1.0 : 0.0, 0.0};
        // S = [[Z, X - iY], [X + iY, -Z]];  A = 1 - ck S
        a[6 * r + c] = one - ck * Z;
        a[6 * r + 3 + c] = -ck * (X - times_i(Y));
        a[6 * (3 + r) + c] = -ck * (X + times_i(Y));
        a[6 * (3 + r) + 3 + c] = one + ck * Z;
      }
    store_block<double2>(out.a64[p], s, b, a);
    if (p == 0) {
      store_block<float2>(out.a32_ee, s, b, a);
      store_block<__half2>(out.a16_ee, s, b, a);
    }
    invert6(a);
    store_block<double2>(out.ai64[p], s, b, a);
    if (p == 1) {
      store_block<float2>(out.ai32_oo, s, b, a);
      store_block<__half2>(out.ai16_oo, s, b, a);
    }
  }
}

}  // namespace

void free_clover(lq_ctx* ctx) {
  Clover& c = ctx->clov;
  for (int p = 0; p < 2; ++p) {
    if (c.a64[p]) (void)hipFree(c.a64[p]);
    if (c.ainv64[p]) (void)hipFree(c.ainv64[p]);
    c.a64[p] = c.ainv64[p] = nullptr;
  }
  for (int q = 0; q < 3; ++q) {
    if (q > 0 && c.a_ee[q]) (void)hipFree(c.a_ee[q]);
    if (q > 0 && c.ainv_oo[q]) (void)hipFree(c.ainv_oo[q]);
    c.a_ee[q] = c.ainv_oo[q] = nullptr;
  }
  c.valid = false;
}

void build_clover(lq_ctx* ctx, double kappa, double csw) {
  LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
  Clover& c = ctx->clov;
  const Geo& g = ctx->geo;
  const size_t n = (size_t)g.nblk * SB * 36;
  if (!c.a64[0]) {
    for (int p = 0; p < 2; ++p) {
      LQ_HIP(hipMalloc(&c.a64[p], n * 16));
      LQ_HIP(hipMalloc(&c.ainv64[p], n * 16));
      LQ_HIP(hipMemsetAsync(c.a64[p], 0, n * 16, ctx->cur));
      LQ_HIP(hipMemsetAsync(c.ainv64[p], 0, n * 16, ctx->cur));
    }
    LQ_HIP(hipMalloc(&c.a_ee[1], n * 8));
    LQ_HIP(hipMalloc(&c.ainv_oo[1], n * 8));
    LQ_HIP(hipMalloc(&c.a_ee[2], n * 4));
    LQ_HIP(hipMalloc(&c.ainv_oo[2], n * 4));
    LQ_HIP(hipMemsetAsync(c.a_ee[1], 0, n * 8, ctx->cur));
    LQ_HIP(hipMemsetAsync(c.ainv_oo[1], 0, n * 8, ctx->cur));
    LQ_HIP(hipMemsetAsync(c.a_ee[2], 0, n * 4, ctx->cur));
    LQ_HIP(hipMemsetAsync(c.ainv_oo[2], 0, n * 4, ctx->cur));
  }
  c.a_ee[0] = c.a64[0];
  c.ainv_oo[0] = c.ainv64[1];
  CloverOut o;
  for (int p = 0; p < 2; ++p) {
    o.a64[p] = (double2*)c.a64[p];
    o.ai64[p] = (double2*)c.ainv64[p];
  }
  o.a32_ee = (float2*)c.a_ee[1];
  o.ai32_oo = (float2*)c.ainv_oo[1];
  o.a16_ee = (__half2*)c.a_ee[2];
  o.ai16_oo = (__half2*)c.ainv_oo[2];
  hipLaunchKernelGGL(build_clover_kernel, dim3(grid_for(ctx->V, 128)), dim3(128), 0, ctx->cur,
                     g, (const double2*)ctx->gauge[0], csw * kappa, o, ctx->V);
  LQ_HIP(hipGetLastError());
  c.kappa = kappa;
  c.csw = csw;
  c.valid = true;
  ++c.gen;
  ctx->mr_clov_ok = false;
}

}  // namespace lq
