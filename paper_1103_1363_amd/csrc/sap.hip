// Schwarz alternating procedure (SAP) preconditioner and the flexible GCR
// solver around it (section 5 of the paper: its SAP-FGCR solver).
//
// The lattice is cut into blocks of B0 x B1 x B2 x B3 sites, coloured like a
// checkerboard; every extent holds an even number of blocks, so two blocks
// of one colour never share a face.  One application K eta of the
// preconditioner runs ncy cycles from psi = 0; a cycle, for each colour in
// turn (0 first), takes nmr minimal-residual steps on every block of that
// colour with Dirichlet boundary conditions (hops that leave the block are
// dropped) and then recomputes the residual r = eta - M psi on the whole
// lattice (except after the last colour of the last cycle, where nothing
// reads it).  One workgroup solves one block, in one of three forms: the
// block's residual and its FP32 links copied into LDS once per launch, the
// clover blocks streamed from HBM at every MR step (one site per thread); or
// the residual with the FP16 clover blocks and links all staged in LDS; or
// that, with MR on the even-odd reduced block operator (a pair of sites per
// thread).  Arithmetic is FP32 on full-lattice fields (even half, then odd
// half).
//
// FGCR: right-preconditioned GCR, z_k = K r, w_k = M z_k orthonormalised by
// Gram-Schmidt against the earlier w (classical, applied twice), r -= <w_k, r>
// w_k.  The z_k are kept as K produced them: the Gram-Schmidt coefficients
// and norms form an upper triangle H with M Z = W H, and the correction
// Z H^-1 (<w_k, r>)_k is formed once per cycle (the same iterates as
// transforming every z_k alike, with one pass over the z_k instead of one per
// step).  The recursion restarts every `restart` steps, where the residual is
// recomputed in FP64 and the FP32 correction added to the FP64 solution
// (iterative refinement, as the paper describes).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "dslash_core.h"
#include "lq_internal.h"
#include "reduce.h"

namespace lq {

struct Sap {
  void* a32[2] = {nullptr, nullptr};  // FP32 clover blocks A of each parity
  uint64_t clov_gen = 0;               // clover build they were copied from (0: none)
  void* a16[2] = {nullptr, nullptr};  // FP16 copies (block solves with block_fp16)
  uint64_t clov_gen16 = 0;
  void* r = nullptr;    // residual (FP32 full field)
  void* tmp = nullptr;  // FP32 full field
  std::vector<void*> z, w;                 // FGCR directions (FP32 full fields)
  void* xc = nullptr;   // FP32 correction
  void* r64 = nullptr;  // FP64 full field
  double* part = nullptr;  // dot-product partials
  double* hpart = nullptr; // host copy (pinned)
  void** wdev = nullptr;   // device arrays of the direction pointers (Gram-Schmidt)
  void** zdev = nullptr;
  double* mres = nullptr;  // batched dot products [64][2]
  double* mpart = nullptr; // their workgroup partials [64][G][2], G = gs_groups()
  float2* coef = nullptr;  // Gram-Schmidt coefficients [64]
  float2* hcoef = nullptr; // host staging (pinned)
};

namespace {

constexpr int SBLK = 256;     // workgroup of the full-lattice kernels
constexpr int DOT_BLOCKS = 1024;
constexpr int SAP_MAXV = 512;  // sites per block at most (one per thread)

size_t half_bytes(const lq_ctx* ctx, int prec) { return parity_field_bytes(ctx->geo.nblk, prec); }
template <class P>
Field<P> half_of(const void* full, const lq_ctx* ctx, int p) {
  char* b = const_cast<char*>(reinterpret_cast<const char*>(full));
  return field_at<P>(b + (p ? half_bytes(ctx, P::id) : 0), ctx->geo.nblk);
}

// out_p = A_p psi_p - kappa H psi_{1-p} at the sites of parity p, or
// eta_p minus that (SUB): the full operator M, one parity per launch.
template <class P, bool SUB>
LQ_HOP_KERNEL(P) void sap_m_kernel(Geo g, int p, Field<P> out, Field<P> eta, Field<P> same,
                                   Field<P> other, const typename P::S* __restrict__ gauge,
                                   const typename P::S* __restrict__ acl, typename P::R kappa) {
  using R = typename P::R;
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  C<R> acc[12], x[12], y[12];
  hop_site<false>(g, other, gauge, p, s, acc);
  load_spinor<P>(same, s, x);
  clover_mul<P>(acl, s, x, y);
#pragma unroll
  for (int c = 0; c < 12; ++c) y[c] = y[c] - kappa * acc[c];
  if constexpr (SUB) {
    load_spinor<P>(eta, s, x);
#pragma unroll
    for (int c = 0; c < 12; ++c) y[c] = x[c] - y[c];
  }
  store_spinor<P>(out, s, y);
}

struct SapBlocks {
  int B[4];   // block extents
  int NB[4];  // blocks per direction
  int vb;     // sites per block
};

// One hop of the block operator at block-local site t: the neighbour's
// spinor from LDS (component-major, vb sites), the link from HBM.
template <int MU>
__device__ __forceinline__ void block_hops(const Geo& g, const float2* __restrict__ gauge, int p,
                                           int64_t s, int64_t sback, const float2* rho, int vb,
                                           int t, int stride, bool fwd, bool bwd,
                                           C<float> acc[12]) {
  if (fwd) {
    C<float> v[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 e = rho[c * vb + t + stride];
      v[c] = C<float>{e.x, e.y};
    }
    project<MU, 1>(v, h);
    load_link<P32>(gauge, g.nblk, p, MU, s, u);
    link_mul<false>(u, h, w);
    reconstruct_add<MU, 1>(acc, w);
  }
  if (bwd) {
    C<float> v[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 e = rho[c * vb + t - stride];
      v[c] = C<float>{e.x, e.y};
    }
    project<MU, -1>(v, h);
    load_link<P32>(gauge, g.nblk, 1 - p, MU, sback, u);
    link_mul<true>(u, h, w);
    reconstruct_add<MU, -1>(acc, w);
  }
}

// Rows 0 and 1 of the forward link in direction MU of block site ts, from
// the LDS copy [mu][6][vb], and row 2 rebuilt.
__device__ __forceinline__ void lds_link(const float2* L, int vb, int mu, int ts, C<float> u[9]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float2 e = L[(mu * 6 + c) * vb + ts];
    u[c] = C<float>{e.x, e.y};
  }
  u[6] = conj(u[1] * u[5] - u[2] * u[4]);
  u[7] = conj(u[2] * u[3] - u[0] * u[5]);
  u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

// As block_hops, with the links from the block's LDS copy: the backward hop
// from t uses the forward link of site t - stride.
template <int MU>
__device__ __forceinline__ void block_hops_lds(const float2* rho, const float2* L, int vb, int t,
                                               int stride, bool fwd, bool bwd, C<float> acc[12]) {
  if (fwd) {
    C<float> v[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 e = rho[c * vb + t + stride];
      v[c] = C<float>{e.x, e.y};
    }
    project<MU, 1>(v, h);
    lds_link(L, vb, MU, t, u);
    link_mul<false>(u, h, w);
    reconstruct_add<MU, 1>(acc, w);
  }
  if (bwd) {
    C<float> v[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 e = rho[c * vb + t - stride];
      v[c] = C<float>{e.x, e.y};
    }
    project<MU, -1>(v, h);
    lds_link(L, vb, MU, t - stride, u);
    link_mul<true>(u, h, w);
    reconstruct_add<MU, -1>(acc, w);
  }
}

// nmr MR steps on block blockIdx.x of colour `colour` (blocks of one colour
// numbered with the x block index fastest), from delta = 0 and rho = r on
// the block; psi += delta there.  One thread per site of the block.  CACHE:
// the block's forward links are read once into LDS (after the residual,
// [4][6][vb]) instead of from HBM at every MR step.
template <bool CACHE>
__global__ __launch_bounds__(SAP_MAXV) void sap_mr_kernel(Geo g, SapBlocks sb, int colour, int nmr,
                                                          float kappa, Field<P32> r0, Field<P32> r1,
                                                          Field<P32> psi0, Field<P32> psi1,
                                                          const float2* __restrict__ gauge,
                                                          const float2* __restrict__ a0,
                                                          const float2* __restrict__ a1) {
  extern __shared__ float2 rho[];  // [12][vb]
  __shared__ double tot[3];
  __shared__ double sh[3][16];
  const int t = threadIdx.x;
  const bool on = t < sb.vb;
  const int tt = on ? t : 0;
  // block coordinates: every x row of blocks holds NB0 / 2 of each colour
  const int half = sb.NB[0] >> 1;
  int j = blockIdx.x;
  const int jx = j % half;
  j /= half;
  const int by = j % sb.NB[1];
  j /= sb.NB[1];
  const int bz = j % sb.NB[2];
  const int bt = j / sb.NB[2];
  const int bx = 2 * jx + ((by + bz + bt + colour) & 1);
  int l[4];
  {
    int q = tt;
    l[0] = q % sb.B[0];
    q /= sb.B[0];
    l[1] = q % sb.B[1];
    q /= sb.B[1];
    l[2] = q % sb.B[2];
    l[3] = q / sb.B[2];
  }
  int x[4] = {bx * sb.B[0] + l[0], by * sb.B[1] + l[1], bz * sb.B[2] + l[2], bt * sb.B[3] + l[3]};
  const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  const int64_t s = cb_index(g, x);
  int64_t sback[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = l[mu] > 0 ? y[mu] - 1 : y[mu];  // inside the block whenever used
    sback[mu] = cb_index(g, y);
  }
  const int stride[4] = {1, sb.B[0], sb.B[0] * sb.B[1], sb.B[0] * sb.B[1] * sb.B[2]};
  Field<P32> rf, pf;  // (selected by value: a reference would put the arguments in memory)
  rf.d = p ? r1.d : r0.d;
  rf.norm = nullptr;
  pf.d = p ? psi1.d : psi0.d;
  pf.norm = nullptr;
  const float2* acl = p ? a1 : a0;
  float2* links = rho + 12 * sb.vb;
  if constexpr (CACHE) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
      if (on && l[mu] + 1 < sb.B[mu])
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const C<float> e = ldnt<P32>(gauge, link32_idx(g.nblk, p, mu, s, c));
          links[(mu * 6 + c) * sb.vb + t] = make_float2(e.re, e.im);
        }
  }
  C<float> rt[12], del[12];
  if (on) load_spinor<P32>(rf, s, rt);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    if (!on) rt[c] = C<float>{0.f, 0.f};
    del[c] = C<float>{0.f, 0.f};
    if (on) rho[c * sb.vb + t] = make_float2(rt[c].re, rt[c].im);
  }
  for (int it = 0; it < nmr; ++it) {
    __syncthreads();
    C<float> q[12];
    double v[3] = {0.0, 0.0, 0.0};
    if (on) {
      C<float> acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = C<float>{0.f, 0.f};
      if constexpr (CACHE) {
        block_hops_lds<0>(rho, links, sb.vb, t, stride[0], l[0] + 1 < sb.B[0], l[0] > 0, acc);
        block_hops_lds<1>(rho, links, sb.vb, t, stride[1], l[1] + 1 < sb.B[1], l[1] > 0, acc);
        block_hops_lds<2>(rho, links, sb.vb, t, stride[2], l[2] + 1 < sb.B[2], l[2] > 0, acc);
        block_hops_lds<3>(rho, links, sb.vb, t, stride[3], l[3] + 1 < sb.B[3], l[3] > 0, acc);
      } else {
        block_hops<0>(g, gauge, p, s, sback[0], rho, sb.vb, t, stride[0], l[0] + 1 < sb.B[0], l[0] > 0, acc);
        block_hops<1>(g, gauge, p, s, sback[1], rho, sb.vb, t, stride[1], l[1] + 1 < sb.B[1], l[1] > 0, acc);
        block_hops<2>(g, gauge, p, s, sback[2], rho, sb.vb, t, stride[2], l[2] + 1 < sb.B[2], l[2] > 0, acc);
        block_hops<3>(g, gauge, p, s, sback[3], rho, sb.vb, t, stride[3], l[3] + 1 < sb.B[3], l[3] > 0, acc);
      }
      clover_mul<P32>(acl, s, rt, q);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        q[c] = q[c] - kappa * acc[c];
        v[0] += (double)q[c].re * rt[c].re + (double)q[c].im * rt[c].im;  // <q, rho>
        v[1] += (double)q[c].re * rt[c].im - (double)q[c].im * rt[c].re;
        v[2] += (double)q[c].re * q[c].re + (double)q[c].im * q[c].im;    // <q, q>
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) q[c] = C<float>{0.f, 0.f};
    }
    block_sum<3>(v, sh);  // (its barriers also end every read of rho above)
    if (t == 0) {
      tot[0] = v[0];
      tot[1] = v[1];
      tot[2] = v[2];
    }
    __syncthreads();
    const double qq = tot[2];
    const C<float> al = qq > 0.0 ? C<float>{(float)(tot[0] / qq), (float)(tot[1] / qq)}
                                 : C<float>{0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      del[c] = del[c] + al * rt[c];
      rt[c] = rt[c] - al * q[c];
      if (on) rho[c * sb.vb + t] = make_float2(rt[c].re, rt[c].im);
    }
  }
  if (on) {
    C<float> o[12];
    load_spinor<P32>(pf, s, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = o[c] + del[c];
    store_spinor<P32>(pf, s, o);
  }
}

// ---- block solves with FP16 operator data staged in LDS
// The block's residual (FP32), its clover blocks A (FP16, 36 half2 per site,
// the library's slot order) and its interior forward links (FP16, rows 0
// and 1; links that leave the block are never used) all sit in LDS, so the
// MR steps read no global memory: per site and colour pass the clover and
// the links cross HBM once instead of once per step.  Arithmetic is FP32.
// Interior forward links of direction mu are numbered over the box with
// extent B[mu] - 1 in mu (x fastest), directions one after another, and
// stored component-major: entry c of link i at L16[c * nl + i].

struct SapLinks16 {
  int base[4];  // first link of each direction
  int nl;       // interior forward links of the block
};

inline SapLinks16 sap_links16(const SapBlocks& sb) {
  SapLinks16 k;
  int n = 0;
  for (int mu = 0; mu < 4; ++mu) {
    k.base[mu] = n;
    n += sb.vb / sb.B[mu] * (sb.B[mu] - 1);
  }
  k.nl = n;
  return k;
}

// Index of the interior forward link of direction mu at block coordinates l
// (l[mu] < B[mu] - 1).
__device__ __forceinline__ int sap_link16_idx(const SapBlocks& sb, const SapLinks16& k, int mu,
                                              const int l[4]) {
  int e[4] = {sb.B[0], sb.B[1], sb.B[2], sb.B[3]};
  e[mu] -= 1;
  return k.base[mu] + l[0] + e[0] * (l[1] + e[1] * (l[2] + e[2] * l[3]));
}

__device__ __forceinline__ C<float> h2c(unsigned w) {
  const float2 f = __half22float2(__builtin_bit_cast(__half2, w));
  return C<float>{f.x, f.y};
}

// Rows 0 and 1 of link i from the FP16 LDS copy, row 2 rebuilt (FP32).
__device__ __forceinline__ void lds_link16(const unsigned* L, int nl, int i, C<float> u[9]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) u[c] = h2c(L[c * nl + i]);
  u[6] = conj(u[1] * u[5] - u[2] * u[4]);
  u[7] = conj(u[2] * u[3] - u[0] * u[5]);
  u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

template <int MU>
__device__ __forceinline__ void block_hops16(const float2* rho, const unsigned* L, int nl, int vb,
                                             int t, int stride, int fi, int bi, C<float> acc[12]) {
  if (fi >= 0) {
    C<float> v[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 e = rho[c * vb + t + stride];
      v[c] = C<float>{e.x, e.y};
    }
    project<MU, 1>(v, h);
    lds_link16(L, nl, fi, u);
    link_mul<false>(u, h, w);
    reconstruct_add<MU, 1>(acc, w);
  }
  if (bi >= 0) {
    C<float> v[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 e = rho[c * vb + t - stride];
      v[c] = C<float>{e.x, e.y};
    }
    project<MU, -1>(v, h);
    lds_link16(L, nl, bi, u);
    link_mul<true>(u, h, w);
    reconstruct_add<MU, -1>(acc, w);
  }
}

// y = A x for the site's clover blocks from the FP16 LDS copy [36][vb].
__device__ __forceinline__ void lds_clover16(const unsigned* A, int vb, int t, const C<float> x[12],
                                             C<float> y[12]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    C<float> m[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) m[k] = h2c(A[(18 * b + k) * vb + t]);
    const C<float>* xb = x + 6 * b;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const float d = (r & 1) ? m[r >> 1].im : m[r >> 1].re;
      C<float> a = d * xb[r];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        if (c == r) continue;
        if (r < c)
          a = a + m[3 + tri_idx(r, c)] * xb[c];
        else
          a = a + cmul_conj(m[3 + tri_idx(c, r)], xb[c]);
      }
      y[6 * b + r] = a;
    }
  }
}

// As sap_mr_kernel, with the operator from FP16 links and clover staged in
// LDS (dynamic LDS: residual [12][vb] float2, clover [36][vb] half2, links
// [6][nl] half2).
__global__ __launch_bounds__(SAP_MAXV) void sap_mr16_kernel(
    Geo g, SapBlocks sb, SapLinks16 lk, int colour, int nmr, float kappa, Field<P32> r0,
    Field<P32> r1, Field<P32> psi0, Field<P32> psi1, const __half2* __restrict__ gauge16,
    const __half2* __restrict__ a0, const __half2* __restrict__ a1) {
  extern __shared__ float2 rho[];
  __shared__ double tot[3];
  __shared__ double sh[3][16];
  const int t = threadIdx.x;
  const bool on = t < sb.vb;
  const int tt = on ? t : 0;
  const int half = sb.NB[0] >> 1;
  int j = blockIdx.x;
  const int jx = j % half;
  j /= half;
  const int by = j % sb.NB[1];
  j /= sb.NB[1];
  const int bz = j % sb.NB[2];
  const int bt = j / sb.NB[2];
  const int bx = 2 * jx + ((by + bz + bt + colour) & 1);
  int l[4];
  {
    int q = tt;
    l[0] = q % sb.B[0];
    q /= sb.B[0];
    l[1] = q % sb.B[1];
    q /= sb.B[1];
    l[2] = q % sb.B[2];
    l[3] = q / sb.B[2];
  }
  int x[4] = {bx * sb.B[0] + l[0], by * sb.B[1] + l[1], bz * sb.B[2] + l[2], bt * sb.B[3] + l[3]};
  const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  const int64_t s = cb_index(g, x);
  const int stride[4] = {1, sb.B[0], sb.B[0] * sb.B[1], sb.B[0] * sb.B[1] * sb.B[2]};
  // interior link of each direction at this site (forward) and at the
  // backward neighbour (whose forward link it is); -1 where a hop leaves
  int fi[4], bi[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    fi[mu] = (on && l[mu] + 1 < sb.B[mu]) ? sap_link16_idx(sb, lk, mu, l) : -1;
    int lb[4] = {l[0], l[1], l[2], l[3]};
    lb[mu] -= 1;
    bi[mu] = (on && l[mu] > 0) ? sap_link16_idx(sb, lk, mu, lb) : -1;
  }
  Field<P32> rf, pf;
  rf.d = p ? r1.d : r0.d;
  rf.norm = nullptr;
  pf.d = p ? psi1.d : psi0.d;
  pf.norm = nullptr;
  const unsigned* acl = reinterpret_cast<const unsigned*>(p ? a1 : a0);
  unsigned* A16 = reinterpret_cast<unsigned*>(rho + 12 * sb.vb);
  unsigned* L16 = A16 + 36 * sb.vb;
  if (on) {
#pragma unroll
    for (int k = 0; k < 36; ++k) A16[k * sb.vb + t] = acl[clov_idx(s, k)];
    const unsigned* gl = reinterpret_cast<const unsigned*>(gauge16);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
      if (fi[mu] >= 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) L16[c * lk.nl + fi[mu]] = gl[link16_idx(g.nblk, p, mu, s, c)];
  }
  C<float> rt[12], del[12];
  if (on) load_spinor<P32>(rf, s, rt);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    if (!on) rt[c] = C<float>{0.f, 0.f};
    del[c] = C<float>{0.f, 0.f};
    if (on) rho[c * sb.vb + t] = make_float2(rt[c].re, rt[c].im);
  }
  for (int it = 0; it < nmr; ++it) {
    __syncthreads();
    C<float> q[12];
    double v[3] = {0.0, 0.0, 0.0};
    if (on) {
      C<float> acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = C<float>{0.f, 0.f};
      block_hops16<0>(rho, L16, lk.nl, sb.vb, t, stride[0], fi[0], bi[0], acc);
      block_hops16<1>(rho, L16, lk.nl, sb.vb, t, stride[1], fi[1], bi[1], acc);
      block_hops16<2>(rho, L16, lk.nl, sb.vb, t, stride[2], fi[2], bi[2], acc);
      block_hops16<3>(rho, L16, lk.nl, sb.vb, t, stride[3], fi[3], bi[3], acc);
      lds_clover16(A16, sb.vb, t, rt, q);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        q[c] = q[c] - kappa * acc[c];
        v[0] += (double)q[c].re * rt[c].re + (double)q[c].im * rt[c].im;  // <q, rho>
        v[1] += (double)q[c].re * rt[c].im - (double)q[c].im * rt[c].re;
        v[2] += (double)q[c].re * q[c].re + (double)q[c].im * q[c].im;    // <q, q>
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) q[c] = C<float>{0.f, 0.f};
    }
    block_sum<3>(v, sh);  // (its barriers also end every read of rho above)
    if (t == 0) {
      tot[0] = v[0];
      tot[1] = v[1];
      tot[2] = v[2];
    }
    __syncthreads();
    const double qq = tot[2];
    const C<float> al = qq > 0.0 ? C<float>{(float)(tot[0] / qq), (float)(tot[1] / qq)}
                                 : C<float>{0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      del[c] = del[c] + al * rt[c];
      rt[c] = rt[c] - al * q[c];
      if (on) rho[c * sb.vb + t] = make_float2(rt[c].re, rt[c].im);
    }
  }
  if (on) {
    C<float> o[12];
    load_spinor<P32>(pf, s, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = o[c] + del[c];
    store_spinor<P32>(pf, s, o);
  }
}

// ---- even-odd reduced block solves (the refinement eq. sapmodel counts)
// The block system M_b d = r splits into the block's even and odd sites
// (global parity); MR runs on the Schur operator
//   Mhat_b d_e = A_ee d_e - kappa^2 H_eo^b A_oo^-1 H_oe^b d_e
// (H^b: the hopping term restricted to the block, Dirichlet) with source
// r_e + kappa H_eo^b A_oo^-1 r_o, from d_e = 0, and then
//   d_o = A_oo^-1 (r_o + kappa H_oe^b d_e).
// One thread holds the pair of block sites (2 i, 2 i + 1), x neighbours of
// opposite parity (the x extent of a block is even): it works on the odd
// one in the first half of an MR step (t_o = A_oo^-1 H_oe^b rho_e) and on the
// even one in the second (q_e = A_ee rho_e - kappa^2 H_eo^b t_o), so every
// lane is busy in both.  LDS: rho_e and t_o by pair [12][vb / 2] (FP32),
// the clover table of each site by block site [36][vb] (FP16: A_ee at even
// sites, A_oo^-1 at odd ones), the interior links as in sap_mr16_kernel.

struct EoSite {
  int t;          // block-local site index
  int l[4];       // block-local coordinates
  int64_t s;      // checkerboard index of its parity
  int fi[4], bi[4];  // interior link of the forward hop / of the backward neighbour (-1: none)
  int nf[4], nb[4];  // pair index of the forward / backward neighbour (-1: outside the block)
};

__device__ __forceinline__ EoSite eo_site(const Geo& g, const SapBlocks& sb, const SapLinks16& lk,
                                          const int org[4], int t, bool on) {
  EoSite e;
  e.t = t;
  int q = t;
  e.l[0] = q % sb.B[0];
  q /= sb.B[0];
  e.l[1] = q % sb.B[1];
  q /= sb.B[1];
  e.l[2] = q % sb.B[2];
  e.l[3] = q / sb.B[2];
  int x[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) x[mu] = org[mu] + e.l[mu];
  e.s = cb_index(g, x);
  const int stride[4] = {1, sb.B[0], sb.B[0] * sb.B[1], sb.B[0] * sb.B[1] * sb.B[2]};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const bool f = on && e.l[mu] + 1 < sb.B[mu], b = on && e.l[mu] > 0;
    e.fi[mu] = f ? sap_link16_idx(sb, lk, mu, e.l) : -1;
    int lb[4] = {e.l[0], e.l[1], e.l[2], e.l[3]};
    lb[mu] -= 1;
    e.bi[mu] = b ? sap_link16_idx(sb, lk, mu, lb) : -1;
    e.nf[mu] = f ? (t + stride[mu]) >> 1 : -1;
    e.nb[mu] = b ? (t - stride[mu]) >> 1 : -1;
  }
  return e;
}

// acc += H^b v at site e, v of the other parity stored by pair [12][hb]
template <int MU>
__device__ __forceinline__ void eo_hops(const float2* v, int hb, const unsigned* L, int nl,
                                        const EoSite& e, C<float> acc[12]) {
  if (e.nf[MU] >= 0) {
    C<float> w12[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 z = v[c * hb + e.nf[MU]];
      w12[c] = C<float>{z.x, z.y};
    }
    project<MU, 1>(w12, h);
    lds_link16(L, nl, e.fi[MU], u);
    link_mul<false>(u, h, w);
    reconstruct_add<MU, 1>(acc, w);
  }
  if (e.nb[MU] >= 0) {
    C<float> w12[12], h[6], u[9], w[6];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 z = v[c * hb + e.nb[MU]];
      w12[c] = C<float>{z.x, z.y};
    }
    project<MU, -1>(w12, h);
    lds_link16(L, nl, e.bi[MU], u);
    link_mul<true>(u, h, w);
    reconstruct_add<MU, -1>(acc, w);
  }
}

__device__ __forceinline__ void eo_hop_all(const float2* v, int hb, const unsigned* L, int nl,
                                           const EoSite& e, C<float> acc[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = C<float>{0.f, 0.f};
  eo_hops<0>(v, hb, L, nl, e, acc);
  eo_hops<1>(v, hb, L, nl, e, acc);
  eo_hops<2>(v, hb, L, nl, e, acc);
  eo_hops<3>(v, hb, L, nl, e, acc);
}

__device__ __forceinline__ void eo_store(float2* v, int hb, int i, const C<float> x[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c * hb + i] = make_float2(x[c].re, x[c].im);
}

__global__ __launch_bounds__(SAP_MAXV / 2) void sap_mr16eo_kernel(
    Geo g, SapBlocks sb, SapLinks16 lk, int colour, int nmr, float kappa, Field<P32> r0,
    Field<P32> r1, Field<P32> psi0, Field<P32> psi1, const __half2* __restrict__ gauge16,
    const __half2* __restrict__ aee16, const __half2* __restrict__ aooinv16) {
  extern __shared__ float2 sm[];
  __shared__ double tot[3];
  __shared__ double sh[3][16];
  const int hb = sb.vb >> 1;
  float2* RE = sm;             // [12][hb] rho_e, at the end d_e
  float2* TO = sm + 12 * hb;   // [12][hb] t_o
  unsigned* A16 = reinterpret_cast<unsigned*>(sm + 24 * hb);  // [36][vb]
  unsigned* L16 = A16 + 36 * sb.vb;                            // [6][nl]
  const int i = threadIdx.x;
  const bool on = i < hb;
  const int ii = on ? i : 0;
  const int half = sb.NB[0] >> 1;
  int j = blockIdx.x;
  const int jx = j % half;
  j /= half;
  const int by = j % sb.NB[1];
  j /= sb.NB[1];
  const int bz = j % sb.NB[2];
  const int bt = j / sb.NB[2];
  const int bx = 2 * jx + ((by + bz + bt + colour) & 1);
  const int org[4] = {bx * sb.B[0], by * sb.B[1], bz * sb.B[2], bt * sb.B[3]};
  // the pair (2 i, 2 i + 1): which of the two is even
  const EoSite a = eo_site(g, sb, lk, org, 2 * ii, on);
  const int pa = (org[0] + org[1] + org[2] + org[3] + a.l[0] + a.l[1] + a.l[2] + a.l[3]) & 1;
  const EoSite E = eo_site(g, sb, lk, org, 2 * ii + pa, on);
  const EoSite O = eo_site(g, sb, lk, org, 2 * ii + 1 - pa, on);
  Field<P32> fe, fo, pe, po;
  fe.d = r0.d;
  fo.d = r1.d;
  pe.d = psi0.d;
  po.d = psi1.d;
  fe.norm = fo.norm = pe.norm = po.norm = nullptr;
  if (on) {
    const unsigned* ae = reinterpret_cast<const unsigned*>(aee16);
    const unsigned* ao = reinterpret_cast<const unsigned*>(aooinv16);
#pragma unroll
    for (int k = 0; k < 36; ++k) {
      A16[k * sb.vb + E.t] = ae[clov16_idx(E.s, k)];
      A16[k * sb.vb + O.t] = ao[clov16_idx(O.s, k)];
    }
    const unsigned* gl = reinterpret_cast<const unsigned*>(gauge16);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      if (E.fi[mu] >= 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) L16[c * lk.nl + E.fi[mu]] = gl[link16_idx(g.nblk, 0, mu, E.s, c)];
      if (O.fi[mu] >= 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) L16[c * lk.nl + O.fi[mu]] = gl[link16_idx(g.nblk, 1, mu, O.s, c)];
    }
  }
  C<float> ro[12], rho[12], del[12], w[12], acc[12];
  if (on) {
    load_spinor<P32>(fo, O.s, ro);
    load_spinor<P32>(fe, E.s, rho);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) ro[c] = rho[c] = C<float>{0.f, 0.f};
  }
  __syncthreads();  // clover and links staged
  // source: rho_e = r_e + kappa H_eo^b A_oo^-1 r_o
  if (on) {
    lds_clover16(A16, sb.vb, O.t, ro, w);
    eo_store(TO, hb, i, w);
  }
  __syncthreads();
  if (on) {
    eo_hop_all(TO, hb, L16, lk.nl, E, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = rho[c] + kappa * acc[c];
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) del[c] = C<float>{0.f, 0.f};
  __syncthreads();  // every read of TO above is done
  if (on) eo_store(RE, hb, i, rho);
  const float k2 = kappa * kappa;
  for (int it = 0; it < nmr; ++it) {
    __syncthreads();
    // odd half: t_o = A_oo^-1 H_oe^b rho_e
    if (on) {
      eo_hop_all(RE, hb, L16, lk.nl, O, acc);
      lds_clover16(A16, sb.vb, O.t, acc, w);
      eo_store(TO, hb, i, w);
    }
    __syncthreads();
    // even half: q_e = A_ee rho_e - kappa^2 H_eo^b t_o
    double v[3] = {0.0, 0.0, 0.0};
    C<float> q[12];
    if (on) {
      eo_hop_all(TO, hb, L16, lk.nl, E, acc);
      lds_clover16(A16, sb.vb, E.t, rho, q);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        q[c] = q[c] - k2 * acc[c];
        v[0] += (double)q[c].re * rho[c].re + (double)q[c].im * rho[c].im;  // <q, rho>
        v[1] += (double)q[c].re * rho[c].im - (double)q[c].im * rho[c].re;
        v[2] += (double)q[c].re * q[c].re + (double)q[c].im * q[c].im;      // <q, q>
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) q[c] = C<float>{0.f, 0.f};
    }
    block_sum<3>(v, sh);  // (its barriers also end every read of RE and TO above)
    if (threadIdx.x == 0) {
      tot[0] = v[0];
      tot[1] = v[1];
      tot[2] = v[2];
    }
    __syncthreads();
    const double qq = tot[2];
    const C<float> al = qq > 0.0 ? C<float>{(float)(tot[0] / qq), (float)(tot[1] / qq)}
                                 : C<float>{0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      del[c] = del[c] + al * rho[c];
      rho[c] = rho[c] - al * q[c];
    }
    if (on) eo_store(RE, hb, i, rho);
  }
  // d_o = A_oo^-1 (r_o + kappa H_oe^b d_e)
  __syncthreads();
  if (on) eo_store(RE, hb, i, del);
  __syncthreads();
  if (on) {
    eo_hop_all(RE, hb, L16, lk.nl, O, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = ro[c] + kappa * acc[c];
    lds_clover16(A16, sb.vb, O.t, acc, w);
    C<float> o[12];
    load_spinor<P32>(pe, E.s, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = o[c] + del[c];
    store_spinor<P32>(pe, E.s, o);
    load_spinor<P32>(po, O.s, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = o[c] + w[c];
    store_spinor<P32>(po, O.s, o);
  }
}

// FP64 clover blocks -> FP16
__global__ void sap_a16_kernel(const double2* __restrict__ in, __half2* __restrict__ out,
                               int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = __floats2half2_rn((float)in[i].x, (float)in[i].y);
}

// FP64 clover blocks -> FP32
// (out in the chunked FP32 table layout)
__global__ void sap_a32_kernel(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 v = in[clov32_to_64(i)];
    out[i] = make_float2((float)v.x, (float)v.y);
  }
}

// Entries of a full field that belong to sites (not the padding of the last
// 64-site block of each parity): entry i of parity half h, for the
// component-major FP64 layout (T = double2) or the chunked FP32 one.
template <class T>
__device__ __forceinline__ bool live_entry(int64_t i, int64_t per_half, int64_t vh) {
  const int64_t k = i % per_half;
  const int64_t in_block = std::is_same<T, double2>::value ? (k % SB) : site_in_block32(k);
  return (k / (12 * SB)) * SB + in_block < vh;
}

// partials of <a, b> (re, im) and |b|^2 over the live entries of two full fields
template <class TA, class TB>
__global__ __launch_bounds__(256) void sap_dot_kernel(const TA* __restrict__ a,
                                                      const TB* __restrict__ b, int64_t n,
                                                      int64_t per_half, int64_t vh,
                                                      double* __restrict__ part) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!live_entry<TA>(i, per_half, vh)) continue;
    const double ax = a[i].x, ay = a[i].y, bx = b[i].x, by = b[i].y;
    v[0] += ax * bx + ay * by;
    v[1] += ax * by - ay * bx;
    v[2] += bx * bx + by * by;
  }
  block_partial<3>(v, part);
}

// Batched Gram-Schmidt.  Each thread keeps GS_E entries of x (or y) in
// registers while it runs over the k earlier directions, so every field is
// read once per call.
constexpr int GS_E = 4;

// part[(j G + b) 2 + c] = workgroup b's partial of <V_j, x> (c = re, im)
__global__ __launch_bounds__(256) void sap_mdot_kernel(const float2* const* __restrict__ V, int k,
                                                       const float2* __restrict__ x, int64_t n,
                                                       int64_t per_half, int64_t vh,
                                                       double* __restrict__ part) {
  float2 xv[GS_E];
  int64_t idx[GS_E];
  bool live[GS_E];
#pragma unroll
  for (int e = 0; e < GS_E; ++e) {
    idx[e] = ((int64_t)blockIdx.x * GS_E + e) * 256 + threadIdx.x;
    live[e] = idx[e] < n && live_entry<float2>(idx[e], per_half, vh);
    xv[e] = live[e] ? x[idx[e]] : make_float2(0.f, 0.f);
  }
  for (int j = 0; j < k; ++j) {
    const float2* v = V[j];
    double a[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < GS_E; ++e)
      if (live[e]) {
        const float2 u = v[idx[e]];
        a[0] += (double)u.x * xv[e].x + (double)u.y * xv[e].y;
        a[1] += (double)u.x * xv[e].y - (double)u.y * xv[e].x;
      }
    block_partial_at<2>(a, part, (int64_t)j * gridDim.x + blockIdx.x);
  }
}

// res[2 j + c] = sum over the G workgroup partials (one workgroup per j)
__global__ __launch_bounds__(256) void sap_mdot_fin_kernel(const double* __restrict__ part, int G,
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

// y -= sum_j c_j V_j over the live entries
__global__ __launch_bounds__(256) void sap_maxpy_kernel(float2* __restrict__ y,
                                                        const float2* const* __restrict__ V,
                                                        const float2* __restrict__ c, int k,
                                                        int64_t n, int64_t per_half, int64_t vh) {
  float2 yv[GS_E];
  int64_t idx[GS_E];
  bool live[GS_E];
#pragma unroll
  for (int e = 0; e < GS_E; ++e) {
    idx[e] = ((int64_t)blockIdx.x * GS_E + e) * 256 + threadIdx.x;
    live[e] = idx[e] < n && live_entry<float2>(idx[e], per_half, vh);
    yv[e] = live[e] ? y[idx[e]] : make_float2(0.f, 0.f);
  }
  for (int j = 0; j < k; ++j) {
    const float2 cj = c[j];
    const float2* v = V[j];
#pragma unroll
    for (int e = 0; e < GS_E; ++e)
      if (live[e]) {
        const float2 u = v[idx[e]];
        yv[e].x -= cj.x * u.x - cj.y * u.y;
        yv[e].y -= cj.x * u.y + cj.y * u.x;
      }
  }
#pragma unroll
  for (int e = 0; e < GS_E; ++e)
    if (live[e]) y[idx[e]] = yv[e];
}

// y = ca x + cb y on FP32 entries (complex ca, cb)
__global__ void sap_caxpby_kernel(float2* __restrict__ y, float ar, float ai,
                                  const float2* __restrict__ x, float br, float bi, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 u = x[i], v = y[i];
  y[i] = make_float2(ar * u.x - ai * u.y + br * v.x - bi * v.y,
                     ar * u.y + ai * u.x + br * v.y + bi * v.x);
}

// FP64 -> FP32 and FP64 += FP32, entrywise
// out = s * in, rounded to FP32 (s = 1 / |in| keeps any FP64 magnitude in range)
// (i counts FP32 entries; the FP64 entry of the same site and component is
// flat32_to_64(i))
__global__ void sap_to32_kernel(float2* __restrict__ out, const double2* __restrict__ in,
                                double s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 v = in[flat32_to_64(i)];
    out[i] = make_float2((float)(s * v.x), (float)(s * v.y));
  }
}
// y += s * x
__global__ void sap_add64_kernel(double2* __restrict__ y, const float2* __restrict__ x,
                                 double s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int64_t i64 = flat32_to_64(i);
    double2 v = y[i64];
    v.x += s * (double)x[i].x;
    v.y += s * (double)x[i].y;
    y[i64] = v;
  }
}

int64_t entries(const lq_ctx* ctx) { return 2 * ctx->geo.nblk * SB * 12; }

__global__ void sap_zero_kernel(float2* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float2(0.f, 0.f);
}

void fill_zero(lq_ctx* ctx, void* p, size_t bytes) {
  const int64_t n = (int64_t)(bytes / 8);
  hipLaunchKernelGGL(sap_zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<float2*>(p), n);
  LQ_HIP(hipGetLastError());
}

Sap* sap_state(lq_ctx* ctx) {
  if (!ctx->sap) ctx->sap = new Sap();
  Sap* sp = ctx->sap;
  LQ_CHECK(ctx->clov.valid, LQ_ESTATE, "no clover term set (lq_set_clover or a solve)");
  // clover tables: 36 complex per site (two 6x6 blocks in 18 slots each)
  const int64_t ncl = ctx->geo.nblk * SB * 36;
  if (!sp->a32[0]) {
    for (int p = 0; p < 2; ++p) LQ_HIP(hipMalloc(&sp->a32[p], (size_t)ncl * sizeof(float2)));
    LQ_HIP(hipMalloc(&sp->r, 2 * half_bytes(ctx, LQ_F32)));
    LQ_HIP(hipMalloc(&sp->tmp, 2 * half_bytes(ctx, LQ_F32)));
    LQ_HIP(hipMalloc(&sp->part, DOT_BLOCKS * 3 * sizeof(double)));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&sp->hpart), DOT_BLOCKS * 3 * sizeof(double)));
  }
  if (sp->clov_gen != ctx->clov.gen) {
    for (int p = 0; p < 2; ++p)
      hipLaunchKernelGGL(sap_a32_kernel, dim3(grid_for(ncl, 256)), dim3(256), 0, ctx->cur,
                         reinterpret_cast<const double2*>(ctx->clov.a64[p]),
                         reinterpret_cast<float2*>(sp->a32[p]), ncl);
    LQ_HIP(hipGetLastError());
    sp->clov_gen = ctx->clov.gen;
  }
  return sp;
}

// The FP16 clover copies for block_fp16, rebuilt with every clover build.
void sap_a16(lq_ctx* ctx, Sap* sp) {
  const int64_t ncl = ctx->geo.nblk * SB * 36;
  if (!sp->a16[0])
    for (int p = 0; p < 2; ++p) LQ_HIP(hipMalloc(&sp->a16[p], (size_t)ncl * sizeof(__half2)));
  if (sp->clov_gen16 != ctx->clov.gen) {
    for (int p = 0; p < 2; ++p)
      hipLaunchKernelGGL(sap_a16_kernel, dim3(grid_for(ncl, 256)), dim3(256), 0, ctx->cur,
                         reinterpret_cast<const double2*>(ctx->clov.a64[p]),
                         reinterpret_cast<__half2*>(sp->a16[p]), ncl);
    LQ_HIP(hipGetLastError());
    sp->clov_gen16 = ctx->clov.gen;
  }
}

// out = M in (SUB: out = eta - M in) on full fields of precision P
template <class P, bool SUB>
void full_m(lq_ctx* ctx, void* out, const void* eta, const void* in) {
  const Geo& g = ctx->geo;
  const auto* gauge = reinterpret_cast<const typename P::S*>(ctx->gauge[P::id]);
  for (int p = 0; p < 2; ++p) {
    const void* acl;
    if constexpr (P::id == LQ_F64)
      acl = ctx->clov.a64[p];
    else
      acl = ctx->sap->a32[p];
    hipLaunchKernelGGL((sap_m_kernel<P, SUB>), dim3(grid_for(g.vh, SBLK)), dim3(SBLK), 0,
                       ctx->cur, g, p, half_of<P>(out, ctx, p),
                       half_of<P>(SUB ? eta : in, ctx, p), half_of<P>(in, ctx, p),
                       half_of<P>(in, ctx, 1 - p), gauge,
                       reinterpret_cast<const typename P::S*>(acl),
                       (typename P::R)ctx->clov.kappa);
  }
  LQ_HIP(hipGetLastError());
  const double site = 8 * link_site_bytes(P::id) + clover_site_bytes(P::id) +
                      (SUB ? 4 : 3) * spinor_site_bytes(P::id);
  ctx->bytes += (double)ctx->V * site;
}

// <a, b> and |b|^2 over two full fields (host values)
template <class TA, class TB>
void dot3(lq_ctx* ctx, const void* a, const void* b, double out[3]) {
  Sap* sp = ctx->sap;
  const int64_t n = entries(ctx);
  hipLaunchKernelGGL((sap_dot_kernel<TA, TB>), dim3(DOT_BLOCKS), dim3(256), 0, ctx->cur,
                     reinterpret_cast<const TA*>(a), reinterpret_cast<const TB*>(b), n, n / 2,
                     ctx->geo.vh, sp->part);
  LQ_HIP(hipGetLastError());
  LQ_HIP(hipMemcpyAsync(sp->hpart, sp->part, DOT_BLOCKS * 3 * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->cur));
  LQ_HIP(hipStreamSynchronize(ctx->cur));
  out[0] = out[1] = out[2] = 0.0;
  for (int i = 0; i < DOT_BLOCKS; ++i)
    for (int k = 0; k < 3; ++k) out[k] += sp->hpart[3 * i + k];
}

void caxpby(lq_ctx* ctx, void* y, std::complex<double> a, const void* x, std::complex<double> b) {
  const int64_t n = entries(ctx);
  hipLaunchKernelGGL(sap_caxpby_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<float2*>(y), (float)a.real(), (float)a.imag(),
                     reinterpret_cast<const float2*>(x), (float)b.real(), (float)b.imag(), n);
  LQ_HIP(hipGetLastError());
}

// w -= sum_j <W_j, w> W_j and z -= (the same coefficients) Z_j over the k
// earlier (orthonormal) directions, twice: classical Gram-Schmidt repeated,
// which orthogonalises as well as the modified form at a fraction of the
// launches and passes over memory.
int gs_groups(const lq_ctx* ctx) { return grid_for(entries(ctx), 256 * GS_E); }

// w -= sum_j <w_j, w> w_j over the k earlier directions, classical and
// applied twice; h (k entries) receives the summed coefficients of both
// passes, and z (may be null) is transformed alike.
void gram_schmidt(lq_ctx* ctx, int k, void* w, void* z, std::complex<double>* h) {
  Sap* sp = ctx->sap;
  const int64_t n = entries(ctx);
  const int G = gs_groups(ctx);
  LQ_CHECK(k >= 1 && k <= 64, LQ_EINVAL, "Gram-Schmidt over 1..64 directions");
  for (int j = 0; j < k; ++j) h[j] = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(sap_mdot_kernel, dim3(G), dim3(256), 0, ctx->cur,
                       reinterpret_cast<const float2* const*>(sp->wdev), k,
                       reinterpret_cast<const float2*>(w), n, n / 2, ctx->geo.vh, sp->mpart);
    hipLaunchKernelGGL(sap_mdot_fin_kernel, dim3(k), dim3(256), 0, ctx->cur, sp->mpart, G,
                       sp->mres);
    LQ_HIP(hipGetLastError());
    LQ_HIP(hipMemcpyAsync(sp->hpart, sp->mres, sizeof(double) * 2 * k, hipMemcpyDeviceToHost,
                          ctx->cur));
    LQ_HIP(hipStreamSynchronize(ctx->cur));
    for (int j = 0; j < k; ++j) {
      sp->hcoef[j] = make_float2((float)sp->hpart[2 * j], (float)sp->hpart[2 * j + 1]);
      h[j] += std::complex<double>(sp->hcoef[j].x, sp->hcoef[j].y);
    }
    LQ_HIP(hipMemcpyAsync(sp->coef, sp->hcoef, sizeof(float2) * k, hipMemcpyHostToDevice,
                          ctx->cur));
    const int Gx = grid_for(n, 256 * GS_E);
    hipLaunchKernelGGL(sap_maxpy_kernel, dim3(Gx), dim3(256), 0, ctx->cur,
                       reinterpret_cast<float2*>(w),
                       reinterpret_cast<const float2* const*>(sp->wdev), sp->coef, k, n, n / 2,
                       ctx->geo.vh);
    if (z)
      hipLaunchKernelGGL(sap_maxpy_kernel, dim3(Gx), dim3(256), 0, ctx->cur,
                         reinterpret_cast<float2*>(z),
                         reinterpret_cast<const float2* const*>(sp->zdev), sp->coef, k, n, n / 2,
                         ctx->geo.vh);
    LQ_HIP(hipGetLastError());
  }
}

// y -= sum_j c_j V_j over the k directions of the device pointer array V
// (coefficients staged through the pinned host buffer).
void sap_lincomb_sub(lq_ctx* ctx, void* y, void** V, const std::complex<double>* c, int k) {
  Sap* sp = ctx->sap;
  const int64_t n = entries(ctx);
  LQ_HIP(hipStreamSynchronize(ctx->cur));  // the staging buffer may still be in flight
  for (int j = 0; j < k; ++j)
    sp->hcoef[j] = make_float2((float)c[j].real(), (float)c[j].imag());
  LQ_HIP(hipMemcpyAsync(sp->coef, sp->hcoef, sizeof(float2) * k, hipMemcpyHostToDevice,
                        ctx->cur));
  hipLaunchKernelGGL(sap_maxpy_kernel, dim3(grid_for(n, 256 * GS_E)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<float2*>(y), reinterpret_cast<const float2* const*>(V),
                     sp->coef, k, n, n / 2, ctx->geo.vh);
  LQ_HIP(hipGetLastError());
}

SapBlocks blocks_of(const lq_ctx* ctx, const lq_sap_params& q) {
  SapBlocks sb;
  sb.vb = 1;
  for (int k = 0; k < 4; ++k) {
    const int b = q.block[k], L = ctx->dims[k];
    LQ_CHECK(b >= 1 && L % b == 0 && (L / b) % 2 == 0, LQ_EINVAL,
             "each block extent must divide the lattice extent an even number of times");
    sb.B[k] = b;
    sb.NB[k] = L / b;
    sb.vb *= b;
  }
  LQ_CHECK(sb.vb <= SAP_MAXV, LQ_EINVAL, "a block holds at most 512 sites");
  LQ_CHECK(q.block_fp16 == 0 || q.block_fp16 == 1, LQ_EINVAL, "block_fp16 is 0 or 1");
  LQ_CHECK(q.block_eo == 0 || q.block_eo == 1, LQ_EINVAL, "block_eo is 0 or 1");
  return sb;
}

void sap_apply_impl(lq_ctx* ctx, void* out, const void* in, const lq_sap_params& q) {
  Sap* sp = sap_state(ctx);
  const SapBlocks sb = blocks_of(ctx, q);
  const int ncy = q.ncycles > 0 ? q.ncycles : 5;
  const int nmr = q.nmr > 0 ? q.nmr : 4;
  const size_t f32 = 2 * half_bytes(ctx, LQ_F32);
  const size_t lds = (size_t)sb.vb * 12 * sizeof(float2);
  const size_t lds_cached = lds + (size_t)sb.vb * 24 * sizeof(float2);
  int dev = 0, maxlds = 0;
  LQ_HIP(hipGetDevice(&dev));
  LQ_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  LQ_CHECK(lds + 4096 <= (size_t)maxlds, LQ_EINVAL, "block too large for the workgroup's LDS");
  // LQ_SAP_LDS_LINKS=0 keeps the links in HBM (tests of both kernels)
  const char* env = std::getenv("LQ_SAP_LDS_LINKS");
  const bool cache = lds_cached + 4096 <= (size_t)maxlds && !(env && env[0] == '0');
  const int threads = (sb.vb + 63) / 64 * 64;
  const int nblk_colour = sb.NB[0] * sb.NB[1] * sb.NB[2] * sb.NB[3] / 2;
  const SapLinks16 lk = sap_links16(sb);
  const size_t lds16 = lds + (size_t)sb.vb * 36 * 4 + (size_t)lk.nl * 6 * 4;
  if (q.block_eo) {
    LQ_CHECK(q.block_fp16, LQ_EINVAL, "the even-odd block solver runs on the FP16 staged "
                                      "operator (block_fp16 = 1)");
    LQ_CHECK(sb.B[0] % 2 == 0, LQ_EINVAL, "the even-odd block solver needs an even x extent");
    LQ_CHECK(ctx->clov.a_ee[LQ_F16] && ctx->clov.ainv_oo[LQ_F16], LQ_ESTATE,
             "no FP16 clover tables");
  }
  if (q.block_fp16) {
    LQ_CHECK(lds16 + 1024 <= (size_t)maxlds, LQ_EINVAL,
             "block too large to stage its FP16 clover and links in LDS (block_fp16 = 0 "
             "streams them)");
    LQ_CHECK(ctx->gauge[LQ_F16], LQ_ESTATE, "no FP16 gauge field");
    sap_a16(ctx, sp);
  }
  fill_zero(ctx, out, f32);
  LQ_HIP(hipMemcpyAsync(sp->r, in, f32, hipMemcpyDeviceToDevice, ctx->cur));
  const auto* gauge = reinterpret_cast<const float2*>(ctx->gauge[LQ_F32]);
  const Geo& g = ctx->geo;
  for (int cy = 0; cy < ncy; ++cy)
    for (int c = 0; c < 2; ++c) {
      // the residual after the last colour of the last cycle is never used
      const bool last = cy == ncy - 1 && c == 1;
      if (q.block_fp16 && q.block_eo) {
        hipLaunchKernelGGL(sap_mr16eo_kernel, dim3(nblk_colour), dim3((sb.vb / 2 + 63) / 64 * 64),
                           lds16, ctx->cur, g, sb, lk, c, nmr, (float)ctx->clov.kappa,
                           half_of<P32>(sp->r, ctx, 0), half_of<P32>(sp->r, ctx, 1),
                           half_of<P32>(out, ctx, 0), half_of<P32>(out, ctx, 1),
                           reinterpret_cast<const __half2*>(ctx->gauge[LQ_F16]),
                           reinterpret_cast<const __half2*>(ctx->clov.a_ee[LQ_F16]),
                           reinterpret_cast<const __half2*>(ctx->clov.ainv_oo[LQ_F16]));
        LQ_HIP(hipGetLastError());
        ctx->bytes += ctx->V / 2.0 * (clover_site_bytes(LQ_F16) +
                                      (double)lk.nl / sb.vb * link_site_bytes(LQ_F16) +
                                      3 * spinor_site_bytes(LQ_F32));
        if (!last) full_m<P32, true>(ctx, sp->r, in, out);
        continue;
      }
      if (q.block_fp16) {
        hipLaunchKernelGGL(sap_mr16_kernel, dim3(nblk_colour), dim3(threads), lds16, ctx->cur, g,
                           sb, lk, c, nmr, (float)ctx->clov.kappa, half_of<P32>(sp->r, ctx, 0),
                           half_of<P32>(sp->r, ctx, 1), half_of<P32>(out, ctx, 0),
                           half_of<P32>(out, ctx, 1),
                           reinterpret_cast<const __half2*>(ctx->gauge[LQ_F16]),
                           reinterpret_cast<const __half2*>(sp->a16[0]),
                           reinterpret_cast<const __half2*>(sp->a16[1]));
        LQ_HIP(hipGetLastError());
        // per site of the colour: its FP16 clover blocks and interior links
        // once, the residual read and the solution read and written once
        ctx->bytes += ctx->V / 2.0 * (clover_site_bytes(LQ_F16) +
                                      (double)lk.nl / sb.vb * link_site_bytes(LQ_F16) +
                                      3 * spinor_site_bytes(LQ_F32));
        if (!last) full_m<P32, true>(ctx, sp->r, in, out);
        continue;
      }
      if (cache)
        hipLaunchKernelGGL(sap_mr_kernel<true>, dim3(nblk_colour), dim3(threads), lds_cached,
                           ctx->cur, g, sb, c, nmr, (float)ctx->clov.kappa,
                           half_of<P32>(sp->r, ctx, 0), half_of<P32>(sp->r, ctx, 1),
                           half_of<P32>(out, ctx, 0), half_of<P32>(out, ctx, 1), gauge,
                           reinterpret_cast<const float2*>(sp->a32[0]),
                           reinterpret_cast<const float2*>(sp->a32[1]));
      else
        hipLaunchKernelGGL(sap_mr_kernel<false>, dim3(nblk_colour), dim3(threads), lds, ctx->cur,
                           g, sb, c, nmr, (float)ctx->clov.kappa, half_of<P32>(sp->r, ctx, 0),
                           half_of<P32>(sp->r, ctx, 1), half_of<P32>(out, ctx, 0),
                           half_of<P32>(out, ctx, 1), gauge,
                           reinterpret_cast<const float2*>(sp->a32[0]),
                           reinterpret_cast<const float2*>(sp->a32[1]));
      LQ_HIP(hipGetLastError());
      // per site of the colour: per MR step the clover blocks (and without
      // the LDS copy 8 links), 4 links once with it, and the residual read
      // and the solution read and written once
      ctx->bytes += ctx->V / 2.0 * (nmr * ((cache ? 0 : 8) * link_site_bytes(LQ_F32) +
                                           clover_site_bytes(LQ_F32)) +
                                    (cache ? 4 : 0) * link_site_bytes(LQ_F32) +
                                    3 * spinor_site_bytes(LQ_F32));
      if (!last) full_m<P32, true>(ctx, sp->r, in, out);
    }
}

}  // namespace

void sap_destroy(Sap* sp) {
  if (!sp) return;
  for (void* p : {sp->a32[0], sp->a32[1], sp->a16[0], sp->a16[1], sp->r, sp->tmp, sp->xc,
                  sp->r64, (void*)sp->part,
                  (void*)sp->wdev, (void*)sp->zdev, (void*)sp->mres, (void*)sp->mpart,
                  (void*)sp->coef})
    if (p) (void)hipFree(p);
  if (sp->hcoef) (void)hipHostFree(sp->hcoef);
  for (void* p : sp->z) (void)hipFree(p);
  for (void* p : sp->w) (void)hipFree(p);
  if (sp->hpart) (void)hipHostFree(sp->hpart);
  delete sp;
}

void sap_apply(lq_ctx* ctx, void* out, const void* in, const lq_sap_params& q) {
  sap_apply_impl(ctx, out, in, q);
}

// FGCR with the SAP preconditioner on the full system M x = b (FP64 fields
// x, b on the device); returns true when ||b - M x|| <= tol ||b||.
bool solve_sap(lq_ctx* ctx, void* x, const void* b, double tol, const lq_sap_params& q,
               lq_solve_report* rep) {
  auto t0 = std::chrono::steady_clock::now();
  const double bytes0 = ctx->bytes;
  Sap* sp = sap_state(ctx);
  (void)blocks_of(ctx, q);
  const int m = q.restart > 0 ? q.restart : 16;
  LQ_CHECK(m <= 64, LQ_EINVAL, "restart length above 64");
  const int maxiter = q.maxiter > 0 ? q.maxiter : 2000;
  const size_t f32 = 2 * half_bytes(ctx, LQ_F32), f64 = 2 * half_bytes(ctx, LQ_F64);
  while ((int)sp->z.size() < m) {
    void *z = nullptr, *w = nullptr;
    LQ_HIP(hipMalloc(&z, f32));
    sp->z.push_back(z);
    LQ_HIP(hipMalloc(&w, f32));
    sp->w.push_back(w);
  }
  if (!sp->xc) LQ_HIP(hipMalloc(&sp->xc, f32));
  if (!sp->r64) LQ_HIP(hipMalloc(&sp->r64, f64));
  if (!sp->wdev) {
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&sp->wdev), 64 * sizeof(void*)));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&sp->zdev), 64 * sizeof(void*)));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&sp->mres), 64 * 2 * sizeof(double)));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&sp->mpart),
                     (size_t)64 * gs_groups(ctx) * 2 * sizeof(double)));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&sp->coef), 64 * sizeof(float2)));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&sp->hcoef), 64 * sizeof(float2)));
  }
  LQ_HIP(hipMemcpy(sp->wdev, sp->w.data(), sp->w.size() * sizeof(void*), hipMemcpyHostToDevice));
  LQ_HIP(hipMemcpy(sp->zdev, sp->z.data(), sp->z.size() * sizeof(void*), hipMemcpyHostToDevice));
  const int64_t n = entries(ctx);
  double d[3];
  dot3<double2, double2>(ctx, b, b, d);
  const double bn = std::sqrt(d[2]);
  int iters = 0, restarts = 0;
  double res = 0.0;
  bool conv = false;
  fill_zero(ctx, x, f64);
  if (bn == 0.0) {
    conv = true;
  } else {
    void* rho = sp->tmp;
    // Stall guard: a cycle that takes no step, or kStall restarts in a row
    // that do not halve the best FP64 residual, end the solve unconverged.
    constexpr int kStall = 5;
    double best = INFINITY;
    int stalled = 0;
    for (;;) {
      full_m<P64, true>(ctx, sp->r64, b, x);
      dot3<double2, double2>(ctx, sp->r64, sp->r64, d);
      res = std::sqrt(d[2]) / bn;
      if (res <= tol) {
        conv = true;
        break;
      }
      if (iters >= maxiter || !std::isfinite(res)) break;
      if (res <= 0.5 * best) {
        best = res;
        stalled = 0;
      } else if (++stalled >= kStall) {
        break;
      }
      ++restarts;
      // The FP32 cycle solves for the normalised residual r / |r|, so that
      // residuals far outside FP32's range (tiny or huge sources) still
      // convert; the correction is scaled back by |r| in FP64.
      const double rn = std::sqrt(d[2]);
      hipLaunchKernelGGL(sap_to32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                         reinterpret_cast<float2*>(rho),
                         reinterpret_cast<const double2*>(sp->r64), 1.0 / rn, n);
      LQ_HIP(hipGetLastError());
      fill_zero(ctx, sp->xc, f32);
      // an FP32 cycle is trusted down to about 1e-5 of its start; the last
      // stops at what the FP64 residual still needs (with a margin of 2)
      const double cycle = std::max(1e-5, 0.5 * tol / res);
      const int iters0 = iters;
      // The preconditioned directions z_k stay as K produced them: with H the
      // upper triangle of Gram-Schmidt coefficients (H[j][k], j < k) and the
      // norms (H[k][k]), M Z = W H, so the correction is Z H^-1 alpha, formed
      // once at the end of the cycle instead of transforming every z_k.
      std::vector<std::complex<double>> H((size_t)m * m, 0.0), alpha(m, 0.0), hk(m);
      int kk = 0;
      for (int k = 0; k < m && iters < maxiter; ++k) {
        sap_apply_impl(ctx, sp->z[k], rho, q);
        full_m<P32, false>(ctx, sp->w[k], nullptr, sp->z[k]);
        if (k > 0) gram_schmidt(ctx, k, sp->w[k], nullptr, hk.data());
        dot3<float2, float2>(ctx, sp->w[k], sp->w[k], d);
        const double wn = std::sqrt(d[2]);
        if (!(wn > 0.0) || !std::isfinite(wn)) break;
        for (int j = 0; j < k; ++j) H[(size_t)j * m + k] = hk[j];
        H[(size_t)k * m + k] = wn;
        caxpby(ctx, sp->w[k], 1.0 / wn, sp->w[k], 0.0);
        dot3<float2, float2>(ctx, sp->w[k], rho, d);
        const std::complex<double> al(d[0], d[1]);
        alpha[k] = al;
        caxpby(ctx, rho, -al, sp->w[k], 1.0);
        ++iters;
        kk = k + 1;
        dot3<float2, float2>(ctx, rho, rho, d);
        if (std::sqrt(d[2]) <= cycle) break;
      }
      if (iters == iters0) break;  // breakdown at the cycle's first direction
      // y = H^-1 alpha (back substitution), xc = Z y
      std::vector<std::complex<double>> y(kk), neg(kk);
      for (int i = kk - 1; i >= 0; --i) {
        std::complex<double> t = alpha[i];
        for (int j = i + 1; j < kk; ++j) t -= H[(size_t)i * m + j] * y[j];
        y[i] = t / H[(size_t)i * m + i];
        neg[i] = -y[i];  // the kernel subtracts
      }
      sap_lincomb_sub(ctx, sp->xc, sp->zdev, neg.data(), kk);
      hipLaunchKernelGGL(sap_add64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                         reinterpret_cast<double2*>(x), reinterpret_cast<const float2*>(sp->xc),
                         rn, n);
      LQ_HIP(hipGetLastError());
    }
  }
  LQ_HIP(hipStreamSynchronize(ctx->cur));
  if (rep) {
    *rep = lq_solve_report{};
    rep->iterations = iters;
    rep->reliable_updates = restarts;
    rep->true_residual = res;
    rep->schur_residual = res;
    rep->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->bytes = ctx->bytes - bytes0;
  }
  return conv;
}

// FGMRES with deflated restarting and the SAP preconditioner on the full
// system (FP32 Krylov basis, FP64 solution and restart residuals).
bool solve_sap_dr(lq_ctx* ctx, void* x, const void* b, double tol, const lq_sap_params& q,
                  lq_solve_report* rep) {
  auto t0 = std::chrono::steady_clock::now();
  const double bytes0 = ctx->bytes;
  Sap* sp = sap_state(ctx);
  (void)blocks_of(ctx, q);
  const int m = q.restart > 0 ? q.restart : 70;
  LQ_CHECK(m >= 2 && m <= 128, LQ_EINVAL, "FGMRES-DR Krylov dimension must be 2..128");
  LQ_CHECK(q.deflate > 0 && q.deflate < m && q.deflate <= 32, LQ_EINVAL,
           "deflated vectors must be 1..min(m-1, 32)");
  const int maxiter = q.maxiter > 0 ? q.maxiter : 2000;
  const size_t f64 = 2 * half_bytes(ctx, LQ_F64);
  if (!sp->r64) LQ_HIP(hipMalloc(&sp->r64, f64));
  double d[3];
  dot3<double2, double2>(ctx, b, b, d);
  const double bn = std::sqrt(d[2]);
  fill_zero(ctx, x, f64);
  SolveTally t;
  bool conv = true, brk = false;
  double last2 = 0.0;
  if (bn > 0.0) {
    KrylovSpace S;
    S.n = entries(ctx);
    S.halves = 2;
    S.vh = ctx->geo.vh;
    S.x64 = x;
    S.r64 = sp->r64;
    S.precond = [&](void* z, const void* v) { sap_apply_impl(ctx, z, v, q); };
    S.op = [&](void* w, const void* z) { full_m<P32, false>(ctx, w, nullptr, z); };
    S.residual64 = [&]() {
      full_m<P64, true>(ctx, sp->r64, b, x);
      double e[3];
      dot3<double2, double2>(ctx, sp->r64, sp->r64, e);
      last2 = e[2];
      return e[2];
    };
    conv = fgmres_dr(ctx, S, m, q.deflate, tol * bn, maxiter, t, brk);
  }
  LQ_HIP(hipStreamSynchronize(ctx->cur));
  if (rep) {
    *rep = lq_solve_report{};
    rep->iterations = t.iterations;
    rep->reliable_updates = t.reliable;
    rep->true_residual = bn > 0.0 ? std::sqrt(last2) / bn : 0.0;
    rep->schur_residual = rep->true_residual;
    rep->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->bytes = ctx->bytes - bytes0;
  }
  return conv;
}

}  // namespace lq
