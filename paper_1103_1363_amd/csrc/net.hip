// Learned gauge-covariant preconditioner: a stack of linear layers
//
//   psi_{l+1}(x) = W0 psi_l(x) + sum_mu [ Wp_mu U_mu(x) psi_l(x+mu)
//                                        + Wm_mu U_mu(x-mu)^+ psi_l(x-mu) ],
//
// each W a complex 4x4 matrix on spin (colour-blind, so the layer commutes
// with gauge transformations), with the fermion boundary phase of the
// hopping term on hops across the time boundary.  No bias, no nonlinearity:
// the net is a linear operator N, used on the even-odd system as
// N_e = P_e N E_e (embed an even field with zeros on the odd sites, apply,
// keep the even sites) inside flexible Krylov solvers, which tolerate a
// preconditioner that changes between iterations (section 5 of the paper,
// the flexible outer solver of its SAP preconditioning).
//
// Fields are FP32 full lattices (even half then odd half, site-blocked);
// weights FP32, gradients accumulated in FP64.  Weight index k per layer:
// 0 = W0, 1 + 2 mu = Wp_mu, 2 + 2 mu = Wm_mu; W[s_out * 4 + t_in].
//
// Gradients (Wirtinger convention): for y = sum_k W_k T_k psi and an upstream
// g = dL/dconj(y),  dL/dconj(W_k) = sum_{x, colour} g(x) (T_k psi)(x)^+  and
// dL/dconj(psi) = sum_k T_k^+ W_k^+ g.  Since T_{mu+}^+ = T_{mu-}, the
// adjoint layer is a layer with weights W0^+, Wm_mu^+ (forward hop) and
// Wp_mu^+ (backward hop).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <type_traits>
#include <vector>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "dslash_core.h"
#include "lq_internal.h"
#include "reduce.h"

namespace lq {

constexpr int NET_K = 9;
constexpr int NET_W = NET_K * 16;  // complex weights per layer
constexpr int NET_BLK = 128;

struct Net {
  lq_ctx* ctx = nullptr;
  int L = 0;
  float2* w = nullptr;      // [L][9][16]
  float2* wadj = nullptr;   // adjoint layers [L][9][16]
  float2* m1 = nullptr;     // Adam first moments (re, im)
  float2* m2 = nullptr;     // Adam second moments
  double2* grad = nullptr;  // accumulated dL/dconj(W) [L][9][16]
  double* part = nullptr;   // weight-gradient partials [9][blocks][32]
  int nblk_grad = 0;
  void* act = nullptr;      // (L + 1) full FP32 fields
  void* gbuf[2] = {nullptr, nullptr};
  void* fbuf[2] = {nullptr, nullptr};  // FP16 full fields of the fast path (lazy)
  unsigned* wh = nullptr;   // the applied weight set as FP16 pairs [L][9][16][2]
  int64_t step = 0;
  uint64_t rng = 0x9e3779b97f4a7c15ull;  // shuffle generator of the training batches (seed 0)
  bool adj_ok = false;
};

namespace {

size_t full32(const lq_ctx* ctx) { return 2 * parity_field_bytes(ctx->geo.nblk, LQ_F32); }
char* half32(void* full, const lq_ctx* ctx, int p) {
  return reinterpret_cast<char*>(full) + (p ? parity_field_bytes(ctx->geo.nblk, LQ_F32) : 0);
}

// z += a b and z += conj(a) b as four multiply-adds (the operators on C
// round each product before the sum)
__device__ __forceinline__ void cmac(C<float>& z, C<float> a, C<float> b) {
  z.re = fmaf(a.re, b.re, fmaf(-a.im, b.im, z.re));
  z.im = fmaf(a.re, b.im, fmaf(a.im, b.re, z.im));
}
__device__ __forceinline__ void cmac_conj(C<float>& z, C<float> a, C<float> b) {
  z.re = fmaf(a.re, b.re, fmaf(a.im, b.im, z.re));
  z.im = fmaf(a.re, b.im, fmaf(-a.im, b.re, z.im));
}

// acc[s][a] += c * sum_t W[s][t] v[t][a]  (component index spin * 3 + colour)
__device__ __forceinline__ void spin_mix_add(const C<float>* __restrict__ W, const C<float> v[12],
                                             float c, C<float> acc[12]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const C<float> wst = c * W[s * 4 + t];
#pragma unroll
      for (int a = 0; a < 3; ++a) cmac(acc[s * 3 + a], wst, v[t * 3 + a]);
    }
}

// T psi at site s of parity p for hop (MU, BACK): the neighbour spinor of
// the other parity carried by the link (all four spins), times the time
// boundary phase.  PI: precision of the input field, PL: of the links.
template <int MU, bool BACK, class PI = P32, class PL = P32>
__device__ __forceinline__ void transport(const Geo& g, const Field<PI>& other,
                                          const typename PL::S* __restrict__ gauge, int p,
                                          int64_t s, const int l[4], const int tc[4], int x3,
                                          C<float> w[12]) {
  float sign = 1.f;
  if constexpr (MU == 3) {
    if (g.apt && x3 == (BACK ? 0 : g.L[3] - 1)) sign = -1.f;
  }
  int y[4] = {tc[0] * g.T[0] + l[0], tc[1] * g.T[1] + l[1], tc[2] * g.T[2] + l[2], x3};
  if constexpr (!BACK)
    y[MU] = (y[MU] + 1 == g.L[MU]) ? 0 : y[MU] + 1;
  else
    y[MU] = (y[MU] == 0) ? g.L[MU] - 1 : y[MU] - 1;
  const int64_t sy = cb_index(g, y);
  C<float> v[12];
  sign *= (float)load_raw<PI>(other, sy, v);
  C<float> u[9];
  if constexpr (!BACK)
    load_link<PL>(gauge, g.nblk, p, MU, s, u);
  else
    load_link<PL>(gauge, g.nblk, 1 - p, MU, sy, u);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C<float> z = {0.f, 0.f};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (BACK)
          cmac_conj(z, u[3 * b + a], v[t * 3 + b]);
        else
          cmac(z, u[3 * a + b], v[t * 3 + b]);
      }
      w[t * 3 + a] = sign * z;
    }
}

template <int MU, bool BACK, class PI, class PL>
__device__ __forceinline__ void layer_hop(const Geo& g, const Field<PI>& other,
                                          const typename PL::S* __restrict__ gauge, int p,
                                          int64_t s, const int l[4], const int tc[4], int x3,
                                          const C<float>* __restrict__ W, C<float> acc[12]) {
  C<float> w[12];
  transport<MU, BACK, PI, PL>(g, other, gauge, p, s, l, tc, x3, w);
  spin_mix_add(W + 16 * (BACK ? 2 + 2 * MU : 1 + 2 * MU), w, 1.f, acc);
}

enum { NET_FULL = 0, NET_SELF = 1, NET_HOPS = 2 };

// out (parity p) = layer(in) restricted to parity p; same = in at parity p,
// other = in at parity 1 - p, W = the layer's 9 x 16 complex weights.
// MODE: NET_FULL, NET_SELF (the other parity of the input is zero) or
// NET_HOPS (this parity of the input is zero).  PS, PO, POUT: precisions of
// the two input parities and the output; PL: of the links.
template <class PS, class PO, class POUT, class PL, int MODE>
__global__ __launch_bounds__(NET_BLK) void net_layer_kernel(Geo g, int p, Field<POUT> out,
                                                            Field<PS> same, Field<PO> other,
                                                            const typename PL::S* __restrict__ gauge,
                                                            const float2* __restrict__ W) {
  __shared__ C<float> ws[NET_W];
  for (int i = threadIdx.x; i < NET_W; i += blockDim.x) ws[i] = C<float>{W[i].x, W[i].y};
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.vh) return;
  C<float> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = C<float>{0.f, 0.f};
  if constexpr (MODE != NET_HOPS) {
    C<float> v[12];
    const float sc = (float)load_raw<PS>(same, s, v);
    spin_mix_add(ws, v, sc, acc);
  }
  if constexpr (MODE != NET_SELF) {
    int l[4], tc[4];
    site_local(g, p, s, l, tc);
    const int x3 = tc[3] * g.T[3] + l[3];
    layer_hop<0, false, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<0, true, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<1, false, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<1, true, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<2, false, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<2, true, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<3, false, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
    layer_hop<3, true, PO, PL>(g, other, gauge, p, s, l, tc, x3, ws, acc);
  }
  store_spinor<POUT>(out, s, acc);
}

// ---------------------------------------------------------------- FP16 form
// The solvers' form of a layer multiplies FP16 operands: every complex
// product a b is two v_dot2_f32_f16 (two half products summed into an FP32
// accumulator), with a written as the half pairs (re, -im) and (im, re).
// The neighbour spinor (raw FP16 components without its site scale) is
// carried by the FP16 link, the result rounded to FP16 pairs, mixed over
// spin by the layer's weights (FP16 pairs, read as wave-uniform scalars)
// and added to the FP32 output with the neighbour's scale.  Per hop that is
// 72 + 96 dot products instead of 336 FP32 multiply-adds.
typedef _Float16 nh2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float dot2(unsigned a, unsigned b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(nh2, a), __builtin_bit_cast(nh2, b), c, false);
}
// a.x b.x + a.y b.y alone: the three-operand form with an inline zero (the
// builtin's two-operand form would first copy a zero into the accumulator)
__device__ __forceinline__ float dot2_first(unsigned a, unsigned b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// the same with a wave-uniform a (a scalar register)
__device__ __forceinline__ float dot2_first_u(unsigned a, unsigned b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "s"(a), "v"(b));
  return r;
}
__device__ __forceinline__ unsigned pack_h(float re, float im) {
  return __builtin_bit_cast(unsigned, nh2{(_Float16)re, (_Float16)im});
}
__device__ __forceinline__ C<float> unpack_h(unsigned u) {
  const nh2 h = __builtin_bit_cast(nh2, u);
  return {(float)h.x, (float)h.y};
}
__device__ __forceinline__ unsigned swap_h(unsigned u) { return (u >> 16) | (u << 16); }

// Indices in the FP16 form are 32-bit: a parity of the lattices the library
// accepts has at most 2^24 sites, so the largest element index (a link
// entry) stays below 2^30.
// chunk 0 of site s of an FP32 field in 16-byte units (chunk k at + 64 k)
__device__ __forceinline__ unsigned chunk32_base(unsigned s) { return (s >> 6) * 384u + (s & 63u); }
// element i of an array of T at base, with a 32-bit byte offset (so that the
// load takes the base from scalar registers and only the offset per lane)
template <class T>
__device__ __forceinline__ const T& at32(const T* base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ T& at32(T* base, unsigned i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T));
}
// Rows 0 and 1 of the FP16 link (parity p, direction mu, site ls) as six pairs:
// one 16-byte and one 8-byte streaming load (chunked FP16 link layout: per
// (parity, mu, block) entries 0..3 of the 64 sites, then entries 4, 5).
__device__ __forceinline__ void ld_link16(const unsigned* __restrict__ gauge, unsigned nblk, int p,
                                          int mu, unsigned ls, unsigned u[6]) {
  const unsigned lb = ((unsigned)(p * 4 + mu) * nblk + (ls >> 6)) * 384u;
  const h16x4 a = __builtin_nontemporal_load(&at32(reinterpret_cast<const h16x4*>(gauge + lb), ls & 63u));
  const h16x2 b =
      __builtin_nontemporal_load(&at32(reinterpret_cast<const h16x2*>(gauge + lb + 256u), ls & 63u));
  u[0] = a.x;
  u[1] = a.y;
  u[2] = a.z;
  u[3] = a.w;
  u[4] = b.x;
  u[5] = b.y;
}

// The 12 FP16 pairs of site s of an FP16 field (three 16-byte chunks of four
// pairs, chunk k of a 64-site block contiguous), and back.
__device__ __forceinline__ void ld_pairs16(const unsigned* d, unsigned s, unsigned v[12]) {
  const h16x4* q = reinterpret_cast<const h16x4*>(d);
  const unsigned b = (s >> 6) * 192u + (s & 63u);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const h16x4 w = at32(q, b + 64u * k);
    v[4 * k] = w.x;
    v[4 * k + 1] = w.y;
    v[4 * k + 2] = w.z;
    v[4 * k + 3] = w.w;
  }
}
__device__ __forceinline__ void st_pairs16(unsigned* d, unsigned s, const unsigned v[12]) {
  h16x4* q = reinterpret_cast<h16x4*>(d);
  const unsigned b = (s >> 6) * 192u + (s & 63u);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    at32(q, b + 64u * k) = h16x4{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
}

// The 12 components of site s as FP16 pairs scaled to a largest component
// of 1, and that scale (FP16 fields store exactly this; an FP32 field is
// rounded the same way).
template <class P>
__device__ __forceinline__ float load_h(const Field<P>& f, unsigned s, unsigned v[12]) {
  const unsigned b = chunk32_base(s);
  if constexpr (P::has_norm) {
    ld_pairs16(reinterpret_cast<const unsigned*>(f.d), s, v);
    return at32(f.norm, s);
  } else {
    C<float> x[12];
    const f32x4* q = reinterpret_cast<const f32x4*>(f.d);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const f32x4 w = at32(q, b + 64u * k);
      x[2 * k] = C<float>{w.x, w.y};
      x[2 * k + 1] = C<float>{w.z, w.w};
    }
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(x[c].re), fabsf(x[c].im)));
    const float inv = scale_inv(m);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = pack_h(inv * x[c].re, inv * x[c].im);
    return m;
  }
}

// Store the 12 components of site s (FP16: scaled to a largest component of
// 1, with the scale), as store_spinor with 32-bit indices.
template <class P>
__device__ __forceinline__ void store_h(const Field<P>& f, unsigned s, const C<float> v[12]) {
  const unsigned b = chunk32_base(s);
  if constexpr (P::has_norm) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    at32(f.norm, s) = m;
    const float inv = scale_inv(m);
    unsigned u[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) u[c] = pack_h(inv * v[c].re, inv * v[c].im);
    st_pairs16(reinterpret_cast<unsigned*>(f.d), s, u);
  } else {
    f32x4* q = reinterpret_cast<f32x4*>(f.d);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      at32(q, b + 64u * k) = f32x4{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
  }
}

// acc[s][a] += c sum_t W[s][t] v[t][a], with v as FP16 pairs (re, im) and
// the hop's weights as pairs F[2 (4 s + t)] = (re, -im), F[2 (4 s + t) + 1] = (im, re).
__device__ __forceinline__ void mix_h(const unsigned* __restrict__ F, const unsigned v[12], float c,
                                      C<float> acc[12]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float yr = dot2_first_u(F[8 * s], v[a]);
      float yi = dot2_first_u(F[8 * s + 1], v[a]);
#pragma unroll
      for (int t = 1; t < 4; ++t) {
        yr = dot2(F[2 * (4 * s + t)], v[3 * t + a], yr);
        yi = dot2(F[2 * (4 * s + t) + 1], v[3 * t + a], yi);
      }
      acc[3 * s + a].re = fmaf(c, yr, acc[3 * s + a].re);
      acc[3 * s + a].im = fmaf(c, yi, acc[3 * s + a].im);
    }
}

// The hop (MU, BACK) of site s: the neighbour's raw spinor carried by the
// FP16 link (U, or U^+ backwards) as FP16 pairs w, and the neighbour's scale
// times the boundary phase.
template <int MU, bool BACK, class PI>
__device__ __forceinline__ float transport_h(const Geo& g, const Field<PI>& other,
                                             const unsigned* __restrict__ gauge, int p, unsigned s,
                                             const int l[4], const int tc[4], int x3,
                                             unsigned w[12]) {
  float sign = 1.f;
  if constexpr (MU == 3) {
    if (g.apt && x3 == (BACK ? 0 : g.L[3] - 1)) sign = -1.f;
  }
  int y[4] = {tc[0] * g.T[0] + l[0], tc[1] * g.T[1] + l[1], tc[2] * g.T[2] + l[2], x3};
  if constexpr (!BACK)
    y[MU] = (y[MU] + 1 == g.L[MU]) ? 0 : y[MU] + 1;
  else
    y[MU] = (y[MU] == 0) ? g.L[MU] - 1 : y[MU] - 1;
  const unsigned sy = (unsigned)cb_index(g, y);
  unsigned v[12];
  const float scale = sign * load_h<PI>(other, sy, v);
  const unsigned ls = BACK ? sy : s;
  unsigned u[9];
  ld_link16(gauge, (unsigned)g.nblk, BACK ? 1 - p : p, MU, ls, u);
  {  // row 2 = conj(row 0 x row 1)
    C<float> r[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) r[c] = unpack_h(u[c]);
    const C<float> z6 = conj(r[1] * r[5] - r[2] * r[4]);
    const C<float> z7 = conj(r[2] * r[3] - r[0] * r[5]);
    const C<float> z8 = conj(r[0] * r[4] - r[1] * r[3]);
    u[6] = pack_h(z6.re, z6.im);
    u[7] = pack_h(z7.re, z7.im);
    u[8] = pack_h(z8.re, z8.im);
  }
  // forward: (U v)_a = sum_b u[a][b] v_b: re with (u.re, -u.im), im with (u.im, u.re)
  // backward: (U^+ v)_a = sum_b conj(u[b][a]) v_b: re with (u.re, u.im), im with (-u.im, u.re)
  unsigned fr[9], fi[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    fr[c] = BACK ? u[c] : (u[c] ^ 0x80000000u);
    fi[c] = BACK ? (swap_h(u[c]) ^ 0x00008000u) : swap_h(u[c]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int e0 = BACK ? a : 3 * a;
      float zr = dot2_first(fr[e0], v[3 * t]);
      float zi = dot2_first(fi[e0], v[3 * t]);
#pragma unroll
      for (int b = 1; b < 3; ++b) {
        const int e = BACK ? 3 * b + a : 3 * a + b;
        zr = dot2(fr[e], v[3 * t + b], zr);
        zi = dot2(fi[e], v[3 * t + b], zi);
      }
      w[3 * t + a] = pack_h(zr, zi);
    }
  return scale;
}

template <int MU, bool BACK, class PO>
__device__ __forceinline__ void layer_hop_h(const Geo& g, const Field<PO>& other,
                                            const unsigned* __restrict__ gauge, int p, unsigned s,
                                            const int l[4], const int tc[4], int x3,
                                            const unsigned* __restrict__ F, C<float> acc[12]) {
  unsigned w[12];
  const float c = transport_h<MU, BACK, PO>(g, other, gauge, p, s, l, tc, x3, w);
  mix_h(F + 32 * (BACK ? 2 + 2 * MU : 1 + 2 * MU), w, c, acc);
}

// As net_layer_kernel, in the FP16 form: F = the layer's weights as FP16
// pairs (net_half_forms_kernel), FP16 links.
template <class PS, class PO, class POUT, int MODE>
__global__ __launch_bounds__(NET_BLK) __attribute__((amdgpu_waves_per_eu(4))) void net_layer_h_kernel(Geo g, int p, Field<POUT> out,
                                                              Field<PS> same, Field<PO> other,
                                                              const unsigned* __restrict__ gauge,
                                                              const unsigned* __restrict__ F) {
  const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (unsigned)g.vh) return;
  C<float> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = C<float>{0.f, 0.f};
  if constexpr (MODE != NET_HOPS) {
    unsigned v[12];
    const float sc = load_h<PS>(same, s, v);
    mix_h(F, v, sc, acc);
  }
  if constexpr (MODE != NET_SELF) {
    int l[4], tc[4];
    site_local(g, p, s, l, tc);
    const int x3 = tc[3] * g.T[3] + l[3];
    layer_hop_h<0, false, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<0, true, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<1, false, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<1, true, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<2, false, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<2, true, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<3, false, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
    layer_hop_h<3, true, PO>(g, other, gauge, p, s, l, tc, x3, F, acc);
  }
  store_h<POUT>(out, s, acc);
}

// ---------------------------------------------------------------- matrix-core form
// A layer whose input is FP16 in both parities, on the matrix cores.  The
// output at a site is sum_h W_h T_h over h = 0 (the site's own spinor) and
// the eight hops (h = the weight index: 1 + 2 mu forward, 2 + 2 mu
// backward), T_h the transported spinor (4 spins x 3 colours).  In real
// form, over the 64 sites of a wave and the 3 colours, that is one product
//   Y[(s, re/im)][(site, a)] = sum_(h, t, re/im) A[(s, re/im)][(h, t, re/im)] B[(h, t, re/im)][(site, a)]
// of the 8 x 72 weight matrix and a 72 x 192 block, computed in
// v_mfma_f32_16x16x32_f16 tiles of 4 terms (K = 32) by 16 sites of one
// colour (N = 16); rows 8-15 of A are zero, and so is K beyond the ninth
// term.  Operand layout (lane l, i = l % 16, g = l / 16): A[i][8 g + j],
// B[8 g + j][i] (eight halves per lane), D[4 g + j][i] (j = 0..3).  Row
// (s, re) of A holds the pairs (re, -im) of W_h[s][t] and row (s, im) the
// pairs (im, re): exactly the FP16 weight pairs of the dot-product form.
// Each lane computes the transported spinors of its own site as in
// net_layer_h_kernel, scaled by the ratio of the term's scale to the
// largest of the site's nine scales (so that FP16 holds them), and writes
// them to LDS, from where the lanes read their B operands; the output comes
// back through LDS to one site per lane and is multiplied by that largest
// scale.
constexpr int NET_MBLK = 64;  // one wave per workgroup

typedef _Float16 nh8 __attribute__((ext_vector_type(8)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef unsigned nu4 __attribute__((ext_vector_type(4)));

// Neighbour number of site (l, tc) for hop (MU, BACK) and the hop's
// boundary sign.
template <int MU, bool BACK>
__device__ __forceinline__ unsigned nb_of(const Geo& g, const int l[4], const int tc[4], int x3,
                                          float& sign) {
  sign = 1.f;
  if constexpr (MU == 3) {
    if (g.apt && x3 == (BACK ? 0 : g.L[3] - 1)) sign = -1.f;
  }
  int y[4] = {tc[0] * g.T[0] + l[0], tc[1] * g.T[1] + l[1], tc[2] * g.T[2] + l[2], x3};
  if constexpr (!BACK)
    y[MU] = (y[MU] + 1 == g.L[MU]) ? 0 : y[MU] + 1;
  else
    y[MU] = (y[MU] == 0) ? g.L[MU] - 1 : y[MU] - 1;
  return (unsigned)cb_index(g, y);
}

// The raw FP16 spinor of neighbour sy carried by the FP16 link of hop
// (MU, BACK) from site s: FP16 pairs w (without the neighbour's scale).
template <int MU, bool BACK>
__device__ __forceinline__ void carry_h(const Geo& g, const Field<P16>& other,
                                        const unsigned* __restrict__ gauge, int p, unsigned s,
                                        unsigned sy, unsigned w[12]) {
  unsigned v[12];
  ld_pairs16(reinterpret_cast<const unsigned*>(other.d), sy, v);
  const unsigned ls = BACK ? sy : s;
  unsigned u[9];
  ld_link16(gauge, (unsigned)g.nblk, BACK ? 1 - p : p, MU, ls, u);
  {
    C<float> r[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) r[c] = unpack_h(u[c]);
    const C<float> z6 = conj(r[1] * r[5] - r[2] * r[4]);
    const C<float> z7 = conj(r[2] * r[3] - r[0] * r[5]);
    const C<float> z8 = conj(r[0] * r[4] - r[1] * r[3]);
    u[6] = pack_h(z6.re, z6.im);
    u[7] = pack_h(z7.re, z7.im);
    u[8] = pack_h(z8.re, z8.im);
  }
  unsigned fr[9], fi[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    fr[c] = BACK ? u[c] : (u[c] ^ 0x80000000u);
    fi[c] = BACK ? (swap_h(u[c]) ^ 0x00008000u) : swap_h(u[c]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int e0 = BACK ? a : 3 * a;
      float zr = dot2_first(fr[e0], v[3 * t]);
      float zi = dot2_first(fi[e0], v[3 * t]);
#pragma unroll
      for (int b2 = 1; b2 < 3; ++b2) {
        const int e = BACK ? 3 * b2 + a : 3 * a + b2;
        zr = dot2(fr[e], v[3 * t + b2], zr);
        zi = dot2(fi[e], v[3 * t + b2], zi);
      }
      w[3 * t + a] = pack_h(zr, zi);
    }
}

// Term h of the site in lane `lane`: its FP16 pairs times ratio, into LDS
// slot `slot` as [slot][site][colour][spin].
template <int H>
__device__ __forceinline__ void stage_term(const Geo& g, const Field<P16>& same,
                                           const Field<P16>& other,
                                           const unsigned* __restrict__ gauge, int p, unsigned s,
                                           const unsigned sy[9], float ratio, unsigned* st,
                                           int slot, int lane) {
  unsigned w[12];
  if constexpr (H == 0) {
    ld_pairs16(reinterpret_cast<const unsigned*>(same.d), s, w);
  } else {
    carry_h<(H - 1) / 2, ((H - 1) & 1) != 0>(g, other, gauge, p, s, sy[H], w);
  }
  const nh2 r2 = {(_Float16)ratio, (_Float16)ratio};
  unsigned* dst = st + (slot * NET_MBLK + lane) * 12;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    nu4 q;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      q[t] = __builtin_bit_cast(unsigned, __builtin_bit_cast(nh2, w[3 * t + a]) * r2);
    *reinterpret_cast<nu4*>(dst + 4 * a) = q;
  }
}

template <class POUT>
__global__ __launch_bounds__(NET_MBLK) __attribute__((amdgpu_waves_per_eu(4))) void net_layer_mfma_kernel(Geo g, int p, Field<POUT> out,
                                                                  Field<P16> same, Field<P16> other,
                                                                  const unsigned* __restrict__ gauge,
                                                                  const unsigned* __restrict__ F) {
  __shared__ __align__(16) unsigned st[2 * NET_MBLK * 12];
  const int lane = threadIdx.x;
  const unsigned vh = (unsigned)g.vh;
  const unsigned s0 = blockIdx.x * NET_MBLK + lane;
  const bool valid = s0 < vh;
  const unsigned s = valid ? s0 : vh - 1;  // every lane takes part in the matrix products
  int l[4], tc[4];
  site_local(g, p, s, l, tc);
  const int x3 = tc[3] * g.T[3] + l[3];
  // neighbour numbers and signed scales of the nine terms
  unsigned sy[9];
  float c[9];
  sy[0] = s;
  float sg[9];
  sg[0] = 1.f;
  sy[1] = nb_of<0, false>(g, l, tc, x3, sg[1]);
  sy[2] = nb_of<0, true>(g, l, tc, x3, sg[2]);
  sy[3] = nb_of<1, false>(g, l, tc, x3, sg[3]);
  sy[4] = nb_of<1, true>(g, l, tc, x3, sg[4]);
  sy[5] = nb_of<2, false>(g, l, tc, x3, sg[5]);
  sy[6] = nb_of<2, true>(g, l, tc, x3, sg[6]);
  sy[7] = nb_of<3, false>(g, l, tc, x3, sg[7]);
  sy[8] = nb_of<3, true>(g, l, tc, x3, sg[8]);
  c[0] = at32(same.norm, s);
#pragma unroll
  for (int h = 1; h < 9; ++h) c[h] = sg[h] * at32(other.norm, sy[h]);
  float cmax = 0.f;
#pragma unroll
  for (int h = 0; h < 9; ++h) cmax = fmaxf(cmax, fabsf(c[h]));
  const float rinv = scale_inv(cmax);
  const int gg = lane >> 4, i = lane & 15;
  // D[4 P + q]: colours 2 P + (row / 8) of sites 16 q .. 16 q + 15
  nf4 D[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) D[q] = nf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (k == 0) {
      stage_term<0>(g, same, other, gauge, p, s, sy, c[0] * rinv, st, 0, lane);
      stage_term<1>(g, same, other, gauge, p, s, sy, c[1] * rinv, st, 1, lane);
    } else if (k == 1) {
      stage_term<2>(g, same, other, gauge, p, s, sy, c[2] * rinv, st, 0, lane);
      stage_term<3>(g, same, other, gauge, p, s, sy, c[3] * rinv, st, 1, lane);
    } else if (k == 2) {
      stage_term<4>(g, same, other, gauge, p, s, sy, c[4] * rinv, st, 0, lane);
      stage_term<5>(g, same, other, gauge, p, s, sy, c[5] * rinv, st, 1, lane);
    } else if (k == 3) {
      stage_term<6>(g, same, other, gauge, p, s, sy, c[6] * rinv, st, 0, lane);
      stage_term<7>(g, same, other, gauge, p, s, sy, c[7] * rinv, st, 1, lane);
    } else {
      stage_term<8>(g, same, other, gauge, p, s, sy, c[8] * rinv, st, 0, lane);
    }
    // A operand, lane (gg, i): row i = (colour slot i / 8, spin, re/im) against
    // K block gg = (term slot gg / 2, colour slot gg % 2); zero off the
    // colour diagonal and past the ninth term
    const int ts = gg >> 1, cb = gg & 1;
    const int h = 2 * k + ts;
    nu4 A;
    {
      const bool on = (i >> 3) == cb && h < 9;
      const unsigned* f = F + 32 * (on ? h : 0) + 8 * ((i >> 1) & 3) + (i & 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) A[t] = on ? f[2 * t] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int P = 0; P < 2; ++P)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = 2 * P + cb;
        const bool live = h < 9 && a < 3;
        const unsigned* src = st + (ts * NET_MBLK + 16 * q + i) * 12 + 4 * (a < 3 ? a : 2);
        const nu4 B = live ? *reinterpret_cast<const nu4*>(src) : nu4{0u, 0u, 0u, 0u};
        D[4 * P + q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
            __builtin_bit_cast(nh8, A), __builtin_bit_cast(nh8, B), D[4 * P + q], 0, 0, 0);
      }
    __syncthreads();
  }
  // D[4 P + q], lane (gg, i): rows 4 gg + j = colour 2 P + gg / 2, spin
  // 2 (gg % 2) + j / 2, re/im j % 2, of site 16 q + i  ->  LDS [site][spin * 3 + colour]
  float* o = reinterpret_cast<float*>(st);
#pragma unroll
  for (int P = 0; P < 2; ++P) {
    const int a = 2 * P + (gg >> 1);
    if (a < 3) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float* e = o + ((16 * q + i) * 12 + 2 * (gg & 1) * 3 + a) * 2;
        e[0] = D[4 * P + q][0];
        e[1] = D[4 * P + q][1];
        e[6] = D[4 * P + q][2];  // next spin: 3 components further
        e[7] = D[4 * P + q][3];
      }
    }
  }
  __syncthreads();
  C<float> acc[12];
#pragma unroll
  for (int e = 0; e < 12; ++e)
    acc[e] = C<float>{cmax * o[(lane * 12 + e) * 2], cmax * o[(lane * 12 + e) * 2 + 1]};
  if (valid) store_h<POUT>(out, s, acc);
}

// FP16 pairs of n complex weights: F[2 i] = (re, -im), F[2 i + 1] = (im, re).
__global__ void net_half_forms_kernel(const float2* __restrict__ w, unsigned* __restrict__ F,
                                      int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 v = w[i];
  F[2 * i] = pack_h(v.x, -v.y);
  F[2 * i + 1] = pack_h(v.y, v.x);
}

// Per-workgroup partial of sum_{x in parity p, colour} g(x) (T_k psi)(x)^+
// for k = blockIdx.y: 16 complex as 32 doubles, part[(k * nblocks + b) * 32 + j].
__global__ __launch_bounds__(256) void net_wgrad_kernel(Geo g, int p, Field<P32> up,
                                                        Field<P32> same, Field<P32> other,
                                                        const float2* __restrict__ gauge,
                                                        double* __restrict__ part) {
  __shared__ double sh[32][16];
  const int k = blockIdx.y;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double o[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) o[j] = 0.0;
  if (s < g.vh) {
    C<float> t[12], gv[12];
    if (k == 0) {
      load_raw<P32>(same, s, t);
    } else {
      int l[4], tc[4];
      site_local(g, p, s, l, tc);
      const int x3 = tc[3] * g.T[3] + l[3];
      switch (k) {
        case 1: transport<0, false>(g, other, gauge, p, s, l, tc, x3, t); break;
        case 2: transport<0, true>(g, other, gauge, p, s, l, tc, x3, t); break;
        case 3: transport<1, false>(g, other, gauge, p, s, l, tc, x3, t); break;
        case 4: transport<1, true>(g, other, gauge, p, s, l, tc, x3, t); break;
        case 5: transport<2, false>(g, other, gauge, p, s, l, tc, x3, t); break;
        case 6: transport<2, true>(g, other, gauge, p, s, l, tc, x3, t); break;
        case 7: transport<3, false>(g, other, gauge, p, s, l, tc, x3, t); break;
        default: transport<3, true>(g, other, gauge, p, s, l, tc, x3, t); break;
      }
    }
    load_raw<P32>(up, s, gv);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {  // g[a][c] * conj(t[b][c])
          const C<float> x = gv[a * 3 + c], y = t[b * 3 + c];
          re += (double)x.re * y.re + (double)x.im * y.im;
          im += (double)x.im * y.re - (double)x.re * y.im;
        }
        o[2 * (a * 4 + b)] = re;
        o[2 * (a * 4 + b) + 1] = im;
      }
  }
  block_sum<32>(o, sh);
  if (threadIdx.x == 0) {
    double* dst = part + ((int64_t)k * gridDim.x + blockIdx.x) * 32;
#pragma unroll
    for (int j = 0; j < 32; ++j) dst[j] = o[j];
  }
}

// grad[k][j] += sum over blocks of part[k][block][j]; workgroup k, threads
// (column = tid % 32, lane = tid / 32).
__global__ __launch_bounds__(256) void net_wgrad_finalize(const double* __restrict__ part,
                                                          int nblocks, double2* __restrict__ grad) {
  __shared__ double sh[8][32];
  const int k = blockIdx.x, col = threadIdx.x & 31, lane = threadIdx.x >> 5;
  double t = 0.0;
  for (int b = lane; b < nblocks; b += 8) t += part[((int64_t)k * nblocks + b) * 32 + col];
  sh[lane][col] = t;
  __syncthreads();
  if (threadIdx.x < 32) {
    double tot = 0.0;
    for (int q = 0; q < 8; ++q) tot += sh[q][col];
    double* gd = reinterpret_cast<double*>(grad + k * 16);
    gd[col] += tot;
  }
}

// Adjoint weight sets: W0^+, and forward/backward hop weights swapped and
// conjugate-transposed.
__global__ void net_adjoint_kernel(const float2* __restrict__ w, float2* __restrict__ wa, int L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L * NET_W) return;
  const int l = i / NET_W, r = i % NET_W, k = r / 16, st = r % 16, s = st / 4, t = st % 4;
  const int ks = k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1);
  const float2 v = w[l * NET_W + ks * 16 + t * 4 + s];
  wa[i] = make_float2(v.x, -v.y);
}

// Adam on the real parameters (Re W, Im W) with gradient 2 (Re, Im) dL/dconj(W);
// clears the accumulated gradient.
__global__ void net_adam_kernel(float2* __restrict__ w, float2* __restrict__ m1,
                                float2* __restrict__ m2, double2* __restrict__ grad, int n,
                                float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gr = (float)(2.0 * grad[i].x), gi = (float)(2.0 * grad[i].y);
  float2 a = m1[i], b = m2[i], x = w[i];
  a.x = b1 * a.x + (1.f - b1) * gr;
  a.y = b1 * a.y + (1.f - b1) * gi;
  b.x = b2 * b.x + (1.f - b2) * gr * gr;
  b.y = b2 * b.y + (1.f - b2) * gi * gi;
  x.x -= lr * (a.x / c1) / (sqrtf(b.x / c2) + eps);
  x.y -= lr * (a.y / c1) / (sqrtf(b.y / c2) + eps);
  m1[i] = a;
  m2[i] = b;
  w[i] = x;
  grad[i] = make_double2(0.0, 0.0);
}

// FP32 full-field helpers
__global__ void net_zero_kernel(float4* __restrict__ p, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

void zero_bytes(lq_ctx* ctx, void* p, size_t bytes) {
  const int64_t n4 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(net_zero_kernel, dim3(grid_for(n4, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<float4*>(p), n4);
  LQ_HIP(hipGetLastError());
}

// out = a x + b y on FP32 fields of `bytes` bytes (elementwise; layout-free)
__global__ void net_axpby_kernel(float4* __restrict__ out, float a, const float4* __restrict__ x,
                                 float b, const float4* __restrict__ y, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const float4 u = x[i], v = y[i];
  out[i] = make_float4(a * u.x + b * v.x, a * u.y + b * v.y, a * u.z + b * v.z, a * u.w + b * v.w);
}

void axpby_f32_impl(lq_ctx* ctx, void* out, double a, const void* x, double b, const void* y) {
  const int64_t n4 = (int64_t)(parity_field_bytes(ctx->geo.nblk, LQ_F32) / 16);
  hipLaunchKernelGGL(net_axpby_kernel, dim3(grid_for(n4, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<float4*>(out), (float)a, reinterpret_cast<const float4*>(x),
                     (float)b, reinterpret_cast<const float4*>(y), n4);
  LQ_HIP(hipGetLastError());
}

// y += c x for complex c, elementwise over the complex entries of two
// fields of one parity (FP32 y and x, or FP64 y and FP32 x; i counts FP32
// entries, and an FP64 y takes the entry of the same site and component).
template <class TY>
__global__ void net_caxpy_kernel(TY* __restrict__ y, double cr, double ci,
                                 const float2* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t iy = std::is_same<TY, double2>::value ? flat32_to_64(i) : i;
  const float2 v = x[i];
  TY o = y[iy];
  o.x += (cr * v.x - ci * v.y);
  o.y += (cr * v.y + ci * v.x);
  y[iy] = o;
}

void copy_bytes(lq_ctx* ctx, void* dst, const void* src, size_t bytes) {
  LQ_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->cur));
}

// one layer on full fields: out = layer(in) with weight set W (both parities)
void layer(lq_ctx* ctx, const float2* W, void* out, void* in) {
  const Geo& g = ctx->geo;
  const auto* gauge = reinterpret_cast<const float2*>(ctx->gauge[LQ_F32]);
  for (int p = 0; p < 2; ++p)
    hipLaunchKernelGGL((net_layer_kernel<P32, P32, P32, P32, NET_FULL>),
                       dim3(grid_for(g.vh, NET_BLK)), dim3(NET_BLK), 0, ctx->cur, g, p,
                       field_at<P32>(half32(out, ctx, p), g.nblk),
                       field_at<P32>(half32(in, ctx, p), g.nblk),
                       field_at<P32>(half32(in, ctx, 1 - p), g.nblk), gauge, W);
  LQ_HIP(hipGetLastError());
  // bytes: the input at this site and (reused) at the neighbours, 8 FP32 links, the output
  ctx->bytes += (double)ctx->V * (2.0 * 96 + 8 * 48 + 96);
}

// one parity of a layer in the fast precision set: FP16 links and FP16
// arithmetic, F = the layer's weights as FP16 pairs
template <class PS, class PO, class POUT, int MODE>
void layer_part(lq_ctx* ctx, const unsigned* F, int p, void* out, const void* same,
                const void* other) {
  const Geo& g = ctx->geo;
  const auto* gauge = reinterpret_cast<const unsigned*>(ctx->gauge[LQ_F16]);
  hipLaunchKernelGGL((net_layer_h_kernel<PS, PO, POUT, MODE>), dim3(grid_for(g.vh, NET_BLK)),
                     dim3(NET_BLK), 0, ctx->cur, g, p, field_at<POUT>(out, g.nblk),
                     field_at<PS>(const_cast<void*>(same), g.nblk),
                     field_at<PO>(const_cast<void*>(other), g.nblk), gauge, F);
  LQ_HIP(hipGetLastError());
  double b = spinor_site_bytes(POUT::id);
  if (MODE != NET_HOPS) b += spinor_site_bytes(PS::id);
  if (MODE != NET_SELF) b += spinor_site_bytes(PO::id) + 8 * link_site_bytes(LQ_F16);
  ctx->bytes += (double)g.vh * b;
}

// one parity of a layer with FP16 input in both parities, on the matrix
// cores (net_layer_mfma_kernel)
template <class POUT>
void layer_part_mfma(lq_ctx* ctx, const unsigned* F, int p, void* out, const void* same,
                     const void* other) {
  const Geo& g = ctx->geo;
  const auto* gauge = reinterpret_cast<const unsigned*>(ctx->gauge[LQ_F16]);
  hipLaunchKernelGGL(net_layer_mfma_kernel<POUT>, dim3(grid_for(g.vh, NET_MBLK)), dim3(NET_MBLK),
                     0, ctx->cur, g, p, field_at<POUT>(out, g.nblk),
                     field_at<P16>(const_cast<void*>(same), g.nblk),
                     field_at<P16>(const_cast<void*>(other), g.nblk), gauge, F);
  LQ_HIP(hipGetLastError());
  const double b = spinor_site_bytes(POUT::id) + 2 * spinor_site_bytes(LQ_F16) +
                   8 * link_site_bytes(LQ_F16);
  ctx->bytes += (double)g.vh * b;
}

void ensure_adjoint(Net* n) {
  if (n->adj_ok) return;
  const int tot = n->L * NET_W;
  hipLaunchKernelGGL(net_adjoint_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, n->ctx->cur, n->w,
                     n->wadj, n->L);
  LQ_HIP(hipGetLastError());
  n->adj_ok = true;
}

// full-field forward through all layers, keeping the activations act[0..L];
// act[0] must hold the input
void forward_all(Net* n) {
  lq_ctx* ctx = n->ctx;
  const size_t fb = full32(ctx);
  char* a = reinterpret_cast<char*>(n->act);
  for (int l = 0; l < n->L; ++l) layer(ctx, n->w + l * NET_W, a + (l + 1) * fb, a + l * fb);
}

}  // namespace

Net* net_create(lq_ctx* ctx, int L) {
  LQ_CHECK(L >= 1 && L <= 16, LQ_EINVAL, "a net has 1..16 layers");
  LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
  Net* n = new Net();
  n->ctx = ctx;
  n->L = L;
  try {
    const size_t wb = (size_t)L * NET_W * sizeof(float2);
    LQ_HIP(hipMalloc(&n->w, wb));
    LQ_HIP(hipMalloc(&n->wadj, wb));
    LQ_HIP(hipMalloc(&n->m1, wb));
    LQ_HIP(hipMalloc(&n->m2, wb));
    LQ_HIP(hipMalloc(&n->grad, (size_t)L * NET_W * sizeof(double2)));
    LQ_HIP(hipMalloc(&n->wh, (size_t)L * NET_W * 2 * sizeof(unsigned)));
    LQ_HIP(hipMemset(n->w, 0, wb));
    LQ_HIP(hipMemset(n->m1, 0, wb));
    LQ_HIP(hipMemset(n->m2, 0, wb));
    LQ_HIP(hipMemset(n->grad, 0, (size_t)L * NET_W * sizeof(double2)));
    n->nblk_grad = grid_for(ctx->geo.vh, 256);
    LQ_HIP(hipMalloc(&n->part, (size_t)NET_K * n->nblk_grad * 32 * sizeof(double)));
    const size_t fb = full32(ctx);
    LQ_HIP(hipMalloc(&n->act, (size_t)(L + 1) * fb));
    LQ_HIP(hipMalloc(&n->gbuf[0], fb));
    LQ_HIP(hipMalloc(&n->gbuf[1], fb));
  } catch (...) {
    net_destroy(n);
    throw;
  }
  return n;
}

void net_destroy(Net* n) {
  if (!n) return;
  for (void* p : {(void*)n->w, (void*)n->wadj, (void*)n->wh, (void*)n->m1, (void*)n->m2, (void*)n->grad,
                  (void*)n->part, n->act, n->gbuf[0], n->gbuf[1], n->fbuf[0], n->fbuf[1]})
    if (p) (void)hipFree(p);
  delete n;
}

int net_layers(const Net* n) { return n->L; }
lq_ctx* net_ctx(const Net* n) { return n->ctx; }

void net_set_weights(Net* n, const double* host) {
  std::vector<float2> h((size_t)n->L * NET_W);
  for (size_t i = 0; i < h.size(); ++i) {
    h[i] = make_float2((float)host[2 * i], (float)host[2 * i + 1]);
    LQ_CHECK(std::isfinite(host[2 * i]) && std::isfinite(host[2 * i + 1]), LQ_EINVAL,
             "non-finite weight");
  }
  LQ_HIP(hipMemcpy(n->w, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice));
  LQ_HIP(hipMemset(n->m1, 0, h.size() * sizeof(float2)));
  LQ_HIP(hipMemset(n->m2, 0, h.size() * sizeof(float2)));
  LQ_HIP(hipMemset(n->grad, 0, h.size() * sizeof(double2)));
  n->step = 0;
  n->adj_ok = false;
}

// Neumann start: W0 = 1, Wp_mu = -(kappa / w_l)(1 - gamma_mu),
// Wm_mu = -(kappa / w_l)(1 + gamma_mu), w_l = exp(2 pi i (l + 1) / (L + 1)),
// so that layer l is 1 - (kappa / w_l) H and the net the truncated series
// sum_{n <= L} (kappa H)^n (prod_l (1 - z / w_l) = 1 + z + ... + z^L).
// Gamma matrices of the chiral basis used by the hopping term:
// gamma_mu = [[0, -i sigma], [i sigma, 0]] for mu = 0, 1, 2, [[0, 1], [1, 0]] for mu = 3.
void net_init_neumann(Net* n, double kappa) {
  using cd = std::complex<double>;
  const cd I(0.0, 1.0);
  cd gam[4][4][4] = {};
  const cd sig[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}}, {{0.0, -I}, {I, 0.0}}, {{1.0, 0.0}, {0.0, -1.0}}};
  for (int mu = 0; mu < 4; ++mu)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const cd blk = mu < 3 ? sig[mu][a][b] : cd(a == b ? 1.0 : 0.0);
        gam[mu][a][2 + b] = mu < 3 ? -I * blk : blk;
        gam[mu][2 + a][b] = mu < 3 ? I * blk : blk;
      }
  std::vector<double> h((size_t)n->L * NET_W * 2, 0.0);
  for (int l = 0; l < n->L; ++l) {
    const cd om = std::polar(1.0, 2.0 * M_PI * (l + 1) / (n->L + 1));
    const cd c = -kappa / om;
    for (int s = 0; s < 4; ++s)
      for (int t = 0; t < 4; ++t) {
        const double one = s == t ? 1.0 : 0.0;
        auto put = [&](int k, cd v) {
          const size_t q = (((size_t)l * NET_K + k) * 16 + s * 4 + t) * 2;
          h[q] = v.real();
          h[q + 1] = v.imag();
        };
        put(0, one);
        for (int mu = 0; mu < 4; ++mu) {
          put(1 + 2 * mu, c * (one - gam[mu][s][t]));
          put(2 + 2 * mu, c * (one + gam[mu][s][t]));
        }
      }
  }
  net_set_weights(n, h.data());
}

void net_get_weights(Net* n, double* host) {
  std::vector<float2> h((size_t)n->L * NET_W);
  LQ_HIP(hipStreamSynchronize(n->ctx->cur));
  LQ_HIP(hipMemcpy(h.data(), n->w, h.size() * sizeof(float2), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < h.size(); ++i) {
    host[2 * i] = h[i].x;
    host[2 * i + 1] = h[i].y;
  }
}

void net_get_grad(Net* n, double* host) {
  LQ_HIP(hipStreamSynchronize(n->ctx->cur));
  LQ_HIP(hipMemcpy(host, n->grad, (size_t)n->L * NET_W * sizeof(double2), hipMemcpyDeviceToHost));
}

void net_zero_grad(Net* n) {
  LQ_HIP(hipMemsetAsync(n->grad, 0, (size_t)n->L * NET_W * sizeof(double2), n->ctx->cur));
}

// y_e = N_e x_e (adjoint: N_e^+ x_e) on FP32 even fields
void net_apply_even(Net* n, void* y_e, const void* x_e, bool adjoint) {
  lq_ctx* ctx = n->ctx;
  const size_t hb = parity_field_bytes(ctx->geo.nblk, LQ_F32);
  const size_t fb = full32(ctx);
  if (adjoint) ensure_adjoint(n);
  const float2* W = adjoint ? n->wadj : n->w;
  // ping-pong between two full fields; the adjoint of E_e ... P_e runs the
  // adjoint layers in reverse order
  char* bufs[2] = {reinterpret_cast<char*>(n->gbuf[0]), reinterpret_cast<char*>(n->gbuf[1])};
  copy_bytes(ctx, bufs[0], x_e, hb);
  zero_bytes(ctx, bufs[0] + hb, fb - hb);
  int cur = 0;
  for (int i = 0; i < n->L; ++i) {
    const int l = adjoint ? n->L - 1 - i : i;
    layer(ctx, W + l * NET_W, bufs[1 - cur], bufs[cur]);
    cur = 1 - cur;
  }
  copy_bytes(ctx, y_e, bufs[cur], hb);
}

// One pair's term of the loss, weight * |N_e b - x|^2 / |x|^2, and the
// accumulation of its gradient (FP32 even fields b, x).
double loss_grad_one(Net* n, const void* b, const void* x, double weight) {
  lq_ctx* ctx = n->ctx;
  const Geo& g = ctx->geo;
  const size_t hb = parity_field_bytes(g.nblk, LQ_F32);
  const size_t fb = full32(ctx);
  ensure_adjoint(n);
  char* act = reinterpret_cast<char*>(n->act);
  const auto* gauge = reinterpret_cast<const float2*>(ctx->gauge[LQ_F32]);
  copy_bytes(ctx, act, b, hb);
  zero_bytes(ctx, act + hb, fb - hb);
  forward_all(n);
  char* out = act + (size_t)n->L * fb;
  // upstream gradient: E_e (y_e - x) weight / |x|^2, held in gbuf[0]
  char* up = reinterpret_cast<char*>(n->gbuf[0]);
  double xn = 0.0, dn = 0.0;
  norm2(ctx, &xn, x, LQ_F32);
  LQ_CHECK(xn > 0.0, LQ_EINVAL, "zero training target");
  axpby_f32_impl(ctx, up, 1.0, out, -1.0, x);
  norm2(ctx, &dn, up, LQ_F32);
  axpby_f32_impl(ctx, up, weight / xn, up, 0.0, up);
  zero_bytes(ctx, up + hb, fb - hb);
  // backward through the layers
  int cur = 0;
  for (int l = n->L - 1; l >= 0; --l) {
    char* gl = reinterpret_cast<char*>(n->gbuf[cur]);
    char* al = act + (size_t)l * fb;
    for (int p = 0; p < 2; ++p) {
      hipLaunchKernelGGL(net_wgrad_kernel, dim3(n->nblk_grad, NET_K), dim3(256), 0, ctx->cur, g,
                         p, field_at<P32>(half32(gl, ctx, p), g.nblk),
                         field_at<P32>(half32(al, ctx, p), g.nblk),
                         field_at<P32>(half32(al, ctx, 1 - p), g.nblk), gauge, n->part);
      hipLaunchKernelGGL(net_wgrad_finalize, dim3(NET_K), dim3(256), 0, ctx->cur, n->part,
                         n->nblk_grad, n->grad + l * NET_W);
    }
    LQ_HIP(hipGetLastError());
    if (l > 0) {
      layer(ctx, n->wadj + l * NET_W, n->gbuf[1 - cur], gl);
      cur = 1 - cur;
    }
  }
  return weight * dn / xn;
}

// y_e = N_e x_e (adjoint: N_e^+ x_e) in the fast precision set used inside
// the solvers: FP16 links, FP16 activations with per-site scales, FP32
// input and output.  The first layer sees an even-only input (its even
// output is W0 x_e alone, its odd output the hops of x_e alone) and only the
// even output of the last layer is formed.
void net_apply_even_fast(Net* n, void* y_e, const void* x_e, bool adjoint) {
  lq_ctx* ctx = n->ctx;
  const size_t h16 = parity_field_bytes(ctx->geo.nblk, LQ_F16);
  if (!n->fbuf[0]) {
    LQ_HIP(hipMalloc(&n->fbuf[0], 2 * h16));
    LQ_HIP(hipMalloc(&n->fbuf[1], 2 * h16));
  }
  if (adjoint) ensure_adjoint(n);
  const int tot = n->L * NET_W;
  hipLaunchKernelGGL(net_half_forms_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, ctx->cur,
                     adjoint ? n->wadj : n->w, n->wh, tot);
  LQ_HIP(hipGetLastError());
  auto wl = [&](int i) { return n->wh + (adjoint ? n->L - 1 - i : i) * NET_W * 2; };
  char* f[2][2] = {{reinterpret_cast<char*>(n->fbuf[0]), reinterpret_cast<char*>(n->fbuf[0]) + h16},
                   {reinterpret_cast<char*>(n->fbuf[1]), reinterpret_cast<char*>(n->fbuf[1]) + h16}};
  if (n->L == 1) {
    layer_part<P32, P32, P32, NET_SELF>(ctx, wl(0), LQ_EVEN, y_e, x_e, x_e);
    return;
  }
  layer_part<P32, P32, P16, NET_SELF>(ctx, wl(0), LQ_EVEN, f[0][0], x_e, x_e);
  layer_part<P32, P32, P16, NET_HOPS>(ctx, wl(0), LQ_ODD, f[0][1], x_e, x_e);
  int cur = 0;
  for (int i = 1; i < n->L - 1; ++i) {
    for (int p = 0; p < 2; ++p)
      layer_part_mfma<P16>(ctx, wl(i), p, f[1 - cur][p], f[cur][p], f[cur][1 - p]);
    cur = 1 - cur;
  }
  layer_part_mfma<P32>(ctx, wl(n->L - 1), LQ_EVEN, y_e, f[cur][0], f[cur][1]);
}

// Loss mean_i |N_e b_i - x_i|^2 / |x_i|^2 over npairs pairs of FP32 even
// fields (npairs consecutive fields each); the gradient of this loss
// replaces the accumulated one.
double net_loss_grad(Net* n, const void* b, const void* x, int npairs) {
  LQ_CHECK(npairs >= 1, LQ_EINVAL, "no pairs");
  const size_t hb = parity_field_bytes(n->ctx->geo.nblk, LQ_F32);
  net_zero_grad(n);
  double loss = 0.0;
  for (int i = 0; i < npairs; ++i)
    loss += loss_grad_one(n, reinterpret_cast<const char*>(b) + (size_t)i * hb,
                          reinterpret_cast<const char*>(x) + (size_t)i * hb, 1.0 / npairs);
  return loss;
}

void net_adam(Net* n, double lr, double b1, double b2, double eps) {
  n->step += 1;
  const int tot = n->L * NET_W;
  const float c1 = (float)(1.0 - std::pow(b1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow(b2, (double)n->step));
  hipLaunchKernelGGL(net_adam_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, n->ctx->cur, n->w,
                     n->m1, n->m2, n->grad, tot, (float)lr, (float)b1, (float)b2, (float)eps, c1,
                     c2);
  LQ_HIP(hipGetLastError());
  n->adj_ok = false;
}

// Training: epochs over npairs (b, x) FP32 even fields in shuffled batches
// (a fixed-seed permutation per epoch), one Adam step per batch; returns the
// mean loss of each epoch in hist (nullable).
void net_train(Net* n, const void* b, const void* x, int npairs, int epochs, int batch, double lr,
               unsigned seed, double* hist) {
  LQ_CHECK(npairs >= 1 && epochs >= 1 && batch >= 1, LQ_EINVAL, "bad training sizes");
  lq_ctx* ctx = n->ctx;
  const size_t hb = parity_field_bytes(ctx->geo.nblk, LQ_F32);
  std::vector<int> perm(npairs);
  for (int i = 0; i < npairs; ++i) perm[i] = i;
  // seed 0 continues the generator where the last training (or the
  // checkpoint it was loaded from) left it
  if (seed != 0) n->rng = 0x9e3779b97f4a7c15ull ^ seed;
  uint64_t& st = n->rng;
  auto rnd = [&st]() {  // splitmix64
    st += 0x9e3779b97f4a7c15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  };
  net_zero_grad(n);
  for (int e = 0; e < epochs; ++e) {
    // each epoch's order depends on the generator state alone (a
    // checkpoint then resumes it exactly)
    for (int i = 0; i < npairs; ++i) perm[i] = i;
    for (int i = npairs - 1; i > 0; --i) std::swap(perm[i], perm[(int)(rnd() % (uint64_t)(i + 1))]);
    double tot = 0.0;
    for (int s0 = 0; s0 < npairs; s0 += batch) {
      const int nb = std::min(batch, npairs - s0);
      double bl = 0.0;
      for (int j = 0; j < nb; ++j) {
        const int q = perm[s0 + j];
        bl += loss_grad_one(n, reinterpret_cast<const char*>(b) + (size_t)q * hb,
                            reinterpret_cast<const char*>(x) + (size_t)q * hb, 1.0 / nb);
      }
      if (!std::isfinite(bl)) throw Error(LQ_ENAN, "non-finite training loss");
      net_adam(n, lr, 0.9, 0.999, 1e-8);
      tot += bl * nb;
    }
    if (hist) hist[e] = tot / npairs;
  }
}

// Checkpoint: one line of JSON (format, version, layers, Adam step, shuffle
// generator state, byte counts), then the FP32 weights and the two Adam
// moment arrays as stored on the device ([L][9][16] (re, im) each), so that
// training resumed from it continues exactly as if it had not stopped.
void net_save(Net* n, const char* path) {
  LQ_CHECK(path && *path, LQ_EINVAL, "no checkpoint path");
  const size_t cnt = (size_t)n->L * NET_W;
  std::vector<float2> w(cnt), m1(cnt), m2(cnt);
  LQ_HIP(hipStreamSynchronize(n->ctx->cur));
  LQ_HIP(hipMemcpy(w.data(), n->w, cnt * sizeof(float2), hipMemcpyDeviceToHost));
  LQ_HIP(hipMemcpy(m1.data(), n->m1, cnt * sizeof(float2), hipMemcpyDeviceToHost));
  LQ_HIP(hipMemcpy(m2.data(), n->m2, cnt * sizeof(float2), hipMemcpyDeviceToHost));
  char head[512];
  std::snprintf(head, sizeof head,
                "{\"format\": \"lq-net-checkpoint\", \"version\": 1, \"layers\": %d, "
                "\"adam_step\": %lld, \"shuffle_state\": \"%016llx\", \"arrays\": "
                "[\"weights\", \"adam_m\", \"adam_v\"], \"bytes_per_array\": %zu, "
                "\"dtype\": \"float32 (re, im) pairs, little endian\"}\n",
                n->L, (long long)n->step, (unsigned long long)n->rng, cnt * sizeof(float2));
  FILE* f = std::fopen(path, "wb");
  LQ_CHECK(f != nullptr, LQ_EINVAL, std::string("cannot write ") + path);
  bool ok = std::fputs(head, f) >= 0;
  for (const auto* v : {&w, &m1, &m2})
    ok = ok && std::fwrite(v->data(), sizeof(float2), cnt, f) == cnt;
  ok = (std::fclose(f) == 0) && ok;
  LQ_CHECK(ok, LQ_EINVAL, std::string("write failed: ") + path);
}

namespace {
// the value after "key": in a one-line JSON object (numbers and strings)
std::string json_field(const std::string& j, const std::string& key) {
  const size_t k = j.find("\"" + key + "\"");
  if (k == std::string::npos) return "";
  size_t c = j.find(':', k);
  if (c == std::string::npos) return "";
  ++c;
  while (c < j.size() && (j[c] == ' ' || j[c] == '"')) ++c;
  size_t e = c;
  while (e < j.size() && j[e] != ',' && j[e] != '"' && j[e] != '}') ++e;
  return j.substr(c, e - c);
}
}  // namespace

void net_load(Net* n, const char* path) {
  LQ_CHECK(path && *path, LQ_EINVAL, "no checkpoint path");
  FILE* f = std::fopen(path, "rb");
  LQ_CHECK(f != nullptr, LQ_EINVAL, std::string("cannot read ") + path);
  std::string head;
  for (int c; (c = std::fgetc(f)) != EOF && c != '\n' && head.size() < 4096;) head.push_back((char)c);
  const size_t cnt = (size_t)n->L * NET_W;
  std::vector<float2> w(cnt), m1(cnt), m2(cnt);
  bool ok = json_field(head, "format") == "lq-net-checkpoint" && json_field(head, "version") == "1";
  const std::string layers = json_field(head, "layers"), step = json_field(head, "adam_step"),
                    rng = json_field(head, "shuffle_state"),
                    bytes = json_field(head, "bytes_per_array");
  if (!ok || layers.empty() || step.empty() || rng.empty() || bytes.empty()) {
    std::fclose(f);
    throw Error(LQ_EINVAL, std::string("not an lq net checkpoint: ") + path);
  }
  if (std::atoi(layers.c_str()) != n->L || std::strtoull(bytes.c_str(), nullptr, 10) !=
                                               cnt * sizeof(float2)) {
    std::fclose(f);
    throw Error(LQ_EINVAL, "checkpoint has another number of layers");
  }
  for (auto* v : {&w, &m1, &m2}) ok = ok && std::fread(v->data(), sizeof(float2), cnt, f) == cnt;
  std::fclose(f);
  LQ_CHECK(ok, LQ_EINVAL, std::string("checkpoint truncated: ") + path);
  for (const float2& z : w)
    LQ_CHECK(std::isfinite(z.x) && std::isfinite(z.y), LQ_EINVAL, "non-finite weight in checkpoint");
  LQ_HIP(hipMemcpy(n->w, w.data(), cnt * sizeof(float2), hipMemcpyHostToDevice));
  LQ_HIP(hipMemcpy(n->m1, m1.data(), cnt * sizeof(float2), hipMemcpyHostToDevice));
  LQ_HIP(hipMemcpy(n->m2, m2.data(), cnt * sizeof(float2), hipMemcpyHostToDevice));
  LQ_HIP(hipMemset(n->grad, 0, cnt * sizeof(double2)));
  n->step = std::strtoll(step.c_str(), nullptr, 10);
  n->rng = std::strtoull(rng.c_str(), nullptr, 16);
  n->adj_ok = false;
}

void caxpy_f32(lq_ctx* ctx, void* y, double cr, double ci, const void* x) {
  const int64_t n = ctx->geo.nblk * SB * 12;
  hipLaunchKernelGGL(net_caxpy_kernel<float2>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<float2*>(y), cr, ci, reinterpret_cast<const float2*>(x), n);
  LQ_HIP(hipGetLastError());
  ctx->bytes += (double)ctx->geo.vh * 3 * 96;
}

void caxpy_64_32(lq_ctx* ctx, void* y64, double cr, double ci, const void* x32) {
  const int64_t n = ctx->geo.nblk * SB * 12;
  hipLaunchKernelGGL(net_caxpy_kernel<double2>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<double2*>(y64), cr, ci, reinterpret_cast<const float2*>(x32),
                     n);
  LQ_HIP(hipGetLastError());
  ctx->bytes += (double)ctx->geo.vh * (2 * 192 + 96);
}

void axpby_f32(lq_ctx* ctx, void* out, double a, const void* x, double b, const void* y) {
  axpby_f32_impl(ctx, out, a, x, b, y);
  ctx->bytes += (double)ctx->geo.vh * 3 * 96;
}

// ---------------------------------------------------------------- Gram-Schmidt
// c_i = <V_i, w> = sum conj(V_i) w for the nv FP32 one-parity fields whose
// device pointers are in V; per-workgroup FP64 partials part[i][block][2].
constexpr int MDOT_BLOCKS = 256;

__global__ __launch_bounds__(256) void multidot_kernel(const float2* const* __restrict__ V,
                                                       const float2* __restrict__ w, int64_t n,
                                                       double* __restrict__ part) {
  __shared__ double sh[2][16];
  const float2* __restrict__ v = V[blockIdx.y];
  double t[2] = {0.0, 0.0};
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const float2 a = v[j], b = w[j];
    t[0] += (double)a.x * b.x + (double)a.y * b.y;
    t[1] += (double)a.x * b.y - (double)a.y * b.x;
  }
  block_sum<2>(t, sh);
  if (threadIdx.x == 0) {
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2] = t[0];
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2 + 1] = t[1];
  }
}

__global__ __launch_bounds__(256) void multidot_finalize(const double* __restrict__ part,
                                                         int nblocks, double* __restrict__ out) {
  __shared__ double sh[2][16];
  double t[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    t[0] += part[((int64_t)blockIdx.x * nblocks + b) * 2];
    t[1] += part[((int64_t)blockIdx.x * nblocks + b) * 2 + 1];
  }
  block_sum<2>(t, sh);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = t[0];
    out[2 * blockIdx.x + 1] = t[1];
  }
}

// w -= sum_i c_i V_i (c: nv complex on the device)
__global__ __launch_bounds__(256) void multiaxpy_kernel(const float2* const* __restrict__ V,
                                                        const double2* __restrict__ c, int nv,
                                                        float2* __restrict__ w, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float2 acc = w[j];
  for (int i = 0; i < nv; ++i) {
    const float2 v = V[i][j];
    const float cr = (float)c[i].x, ci = (float)c[i].y;
    acc.x -= cr * v.x - ci * v.y;
    acc.y -= cr * v.y + ci * v.x;
  }
  w[j] = acc;
}

void multidot_f32(lq_ctx* ctx, const void* vdev, int nv, const void* w, double* part,
                  double* res_dev, double* res_host) {
  const int64_t n = ctx->geo.nblk * SB * 12;
  hipLaunchKernelGGL(multidot_kernel, dim3(MDOT_BLOCKS, nv), dim3(256), 0, ctx->cur,
                     reinterpret_cast<const float2* const*>(vdev),
                     reinterpret_cast<const float2*>(w), n, part);
  hipLaunchKernelGGL(multidot_finalize, dim3(nv), dim3(256), 0, ctx->cur, part, MDOT_BLOCKS,
                     res_dev);
  LQ_HIP(hipGetLastError());
  LQ_HIP(hipMemcpyAsync(res_host, res_dev, sizeof(double) * 2 * nv, hipMemcpyDeviceToHost,
                        ctx->cur));
  LQ_HIP(hipStreamSynchronize(ctx->cur));
  ctx->bytes += (double)ctx->geo.vh * 96.0 * (nv + 1);
}

void multiaxpy_f32(lq_ctx* ctx, const void* vdev, int nv, const double* c_dev, void* w) {
  const int64_t n = ctx->geo.nblk * SB * 12;
  hipLaunchKernelGGL(multiaxpy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur,
                     reinterpret_cast<const float2* const*>(vdev),
                     reinterpret_cast<const double2*>(c_dev), nv, reinterpret_cast<float2*>(w),
                     n);
  LQ_HIP(hipGetLastError());
  ctx->bytes += (double)ctx->geo.vh * 96.0 * (nv + 2);
}

}  // namespace lq
