// Per-site device routines of the even-odd Wilson hopping term and of the
// clover term.  Included by every kernel that applies (part of) the operator.
//
// Hopping term (kappa normalisation, Wilson r = 1):
//   (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)]
// with the chiral-basis gammas of include/lq.h.  Each term is computed as a
// spin projection to a two-spinor h (two colour vectors), a 3x3 link
// product on both colour vectors, and a sign/permutation/i-multiplication
// that rebuilds the lower two spin components from h (no flops).  With
// S = +1 the projector is (1 - gamma_mu), with S = -1 it is (1 + gamma_mu):
//   mu = 0:  h0 = p0 + S i p3,  h1 = p1 + S i p2;  lower: (-S i h1, -S i h0)
//   mu = 1:  h0 = p0 + S p3,    h1 = p1 - S p2;    lower: (-S h1,   +S h0)
//   mu = 2:  h0 = p0 + S i p2,  h1 = p1 - S i p3;  lower: (-S i h0, +S i h1)
//   mu = 3:  h0 = p0 - S p2,    h1 = p1 - S p3;    lower: (-S h0,   -S h1)
// (p_k the colour vector of spin k).  The t-boundary sign is applied here,
// never folded into the links: the third row of a compressed link is
// rebuilt as conj(row0 x row1), which holds only for det U = +1.
#pragma once

#include "lq_internal.h"

// Hops per scheduling group of the hopping kernels (1, 2, 4 or 8).
#ifndef LQ_HOP_GROUP
#define LQ_HOP_GROUP 2
#endif
// FP16 hops on packed halves and dot2 (1) or in FP32 after conversion (0).
#ifndef LQ_HOP16_PACKED
#define LQ_HOP16_PACKED 1
#endif


namespace lq {

// XCD-aware block order: the hardware deals workgroups round-robin to the 8
// XCDs (each with its own L2); this maps them so that each XCD walks one
// contiguous range of logical blocks, keeping neighbouring sites in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7;
  const int64_t k = b & 7, j = b >> 3;
  return k * q + (k < r ? k : r) + j;
}

template <int MU, int S, class R>
__device__ __forceinline__ void project(const C<R> v[12], C<R> h[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const C<R> p0 = v[a], p1 = v[3 + a], p2 = v[6 + a], p3 = v[9 + a];
    if constexpr (MU == 0) {
      h[a] = S > 0 ? p0 + times_i(p3) : p0 - times_i(p3);
      h[3 + a] = S > 0 ? p1 + times_i(p2) : p1 - times_i(p2);
    } else if constexpr (MU == 1) {
      h[a] = S > 0 ? p0 + p3 : p0 - p3;
      h[3 + a] = S > 0 ? p1 - p2 : p1 + p2;
    } else if constexpr (MU == 2) {
      h[a] = S > 0 ? p0 + times_i(p2) : p0 - times_i(p2);
      h[3 + a] = S > 0 ? p1 - times_i(p3) : p1 + times_i(p3);
    } else {
      h[a] = S > 0 ? p0 - p2 : p0 + p2;
      h[3 + a] = S > 0 ? p1 - p3 : p1 + p3;
    }
  }
}

template <int MU, int S, class R>
__device__ __forceinline__ void reconstruct_add(C<R> acc[12], const C<R> w[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const C<R> w0 = w[a], w1 = w[3 + a];
    acc[a] = acc[a] + w0;
    acc[3 + a] = acc[3 + a] + w1;
    if constexpr (MU == 0) {
      acc[6 + a] = S > 0 ? acc[6 + a] - times_i(w1) : acc[6 + a] + times_i(w1);
      acc[9 + a] = S > 0 ? acc[9 + a] - times_i(w0) : acc[9 + a] + times_i(w0);
    } else if constexpr (MU == 1) {
      acc[6 + a] = S > 0 ? acc[6 + a] - w1 : acc[6 + a] + w1;
      acc[9 + a] = S > 0 ? acc[9 + a] + w0 : acc[9 + a] - w0;
    } else if constexpr (MU == 2) {
      acc[6 + a] = S > 0 ? acc[6 + a] - times_i(w0) : acc[6 + a] + times_i(w0);
      acc[9 + a] = S > 0 ? acc[9 + a] + times_i(w1) : acc[9 + a] - times_i(w1);
    } else {
      acc[6 + a] = S > 0 ? acc[6 + a] - w0 : acc[6 + a] + w0;
      acc[9 + a] = S > 0 ? acc[9 + a] - w1 : acc[9 + a] + w1;
    }
  }
}

// Load rows 0 and 1 of a compressed link and rebuild row 2.
template <class P>
__device__ __forceinline__ void load_link(const typename P::S* __restrict__ gauge, int64_t nblk,
                                          int p, int mu, int64_t s, C<typename P::R> u[9]) {
  using R = typename P::R;
  if constexpr (P::id == LQ_F16) {
    unsigned w[6];
    load_link16_raw(gauge, nblk, p, mu, s, w);
#pragma unroll
    for (int c = 0; c < 6; ++c) u[c] = h2_to_c(w[c]);
  } else if constexpr (P::id == LQ_F32) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const f32x4 w = __builtin_nontemporal_load(
          reinterpret_cast<const f32x4*>(gauge + link32_idx(nblk, p, mu, s, 2 * k)));
      u[2 * k] = {w.x, w.y};
      u[2 * k + 1] = {w.z, w.w};
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) u[c] = ldnt<P>(gauge, link_idx(nblk, p, mu, s, c));
  }
  // row2 = conj(row0 x row1)
  u[6] = conj(u[1] * u[5] - u[2] * u[4]);
  u[7] = conj(u[2] * u[3] - u[0] * u[5]);
  u[8] = conj(u[0] * u[4] - u[1] * u[3]);
  (void)sizeof(R);
}

// w = U h (both colour vectors), or U^+ h when DAGU.
template <bool DAGU, class R>
__device__ __forceinline__ void link_mul(const C<R> u[9], const C<R> h[6], C<R> w[6]) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C<R> acc;
      if constexpr (!DAGU) {
        acc = u[3 * a] * h[3 * k];
        acc = acc + u[3 * a + 1] * h[3 * k + 1];
        acc = acc + u[3 * a + 2] * h[3 * k + 2];
      } else {
        acc = cmul_conj(u[a], h[3 * k]);
        acc = acc + cmul_conj(u[3 + a], h[3 * k + 1]);
        acc = acc + cmul_conj(u[6 + a], h[3 * k + 2]);
      }
      w[3 * k + a] = acc;
    }
}

// ---------------------------------------------------------------- FP16 hops
// The FP16 operator keeps the neighbour spinor and the link as half pairs:
// the spin projection is one packed half add per complex component (the
// sum rounds once to FP16, as the stored components already did), and the
// link product runs on v_dot2_f32_f16, two half products summed into an
// FP32 accumulator per instruction.  A complex product u h is
//   Re = dot2(u, (h.re, -h.im)),  Im = dot2(u, (h.im, h.re)),
// and conj(u) h is
//   Re = dot2(u, (h.re, h.im)),   Im = dot2(u, (h.im, -h.re)),
// so the projection produces the two forms of h that the direction needs.
// The third row of the link, conj(row0 x row1), is formed the same way and
// rounded once to FP16.  The neighbour's scale and the accumulation are FP32.
typedef _Float16 hf2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ hf2 hf2_bits(unsigned u) {
  hf2 h;
  __builtin_memcpy(&h, &u, 4);
  return h;
}
__device__ __forceinline__ float dot2(hf2 a, hf2 b, float c) {
  return __builtin_amdgcn_fdot2(a, b, c, false);
}
// c * q for c = +1 (K = 0), -1 (1), +i (2), -i (3)
template <int K>
__device__ __forceinline__ hf2 cmulk(hf2 q) {
  if constexpr (K == 0) return q;
  else if constexpr (K == 1) return hf2{-q.x, -q.y};
  else if constexpr (K == 2) return hf2{-q.y, q.x};
  else return hf2{q.y, -q.x};
}
// h = a + c b in the two forms the link product takes: (re, -im) and
// (im, re) for U h; (re, im) and (im, -re) for U^+ h.
template <int K, bool DAGU>
__device__ __forceinline__ void hform(hf2 a, hf2 b, hf2& f0, hf2& f1) {
  const hf2 q = cmulk<K>(b);
  if constexpr (!DAGU) {
    f0 = hf2{a.x, -a.y} + hf2{q.x, -q.y};
    f1 = hf2{a.y, a.x} + hf2{q.y, q.x};
  } else {
    f0 = a + q;
    f1 = hf2{a.y, -a.x} + hf2{q.y, -q.x};
  }
}
// coefficient codes of the projector (1 - S gamma_mu) in the chiral basis:
// h0 = p0 + c0 p(b0), h1 = p1 + c1 p(b1)
template <int MU, int S>
struct Proj;
template <int S>
struct Proj<0, S> {  // h0 = p0 + S i p3, h1 = p1 + S i p2
  static constexpr int b0 = 3, b1 = 2, k0 = S > 0 ? 2 : 3, k1 = S > 0 ? 2 : 3;
};
template <int S>
struct Proj<1, S> {  // h0 = p0 + S p3, h1 = p1 - S p2
  static constexpr int b0 = 3, b1 = 2, k0 = S > 0 ? 0 : 1, k1 = S > 0 ? 1 : 0;
};
template <int S>
struct Proj<2, S> {  // h0 = p0 + S i p2, h1 = p1 - S i p3
  static constexpr int b0 = 2, b1 = 3, k0 = S > 0 ? 2 : 3, k1 = S > 0 ? 3 : 2;
};
template <int S>
struct Proj<3, S> {  // h0 = p0 - S p2, h1 = p1 - S p3
  static constexpr int b0 = 2, b1 = 3, k0 = S > 0 ? 1 : 0, k1 = S > 0 ? 1 : 0;
};

// STEP: the neighbour's number by the division-free step (fewer
// instructions, but the compiler then computes the numbers of all hops
// early and holds them: 157 instead of 105 registers; right for the plain
// hopping kernel, wrong for the fused solver kernels, which add the clover
// term and the vector updates) or from the neighbour's coordinates.
template <int MU, int S, bool BACK, bool STEP>
__device__ __forceinline__ void hop_dir16(const Geo& g, const Field<P16>& in,
                                          const __half2* __restrict__ gauge, int p, int64_t s,
                                          const int l[4], const int tc[4], int x3, C<float> acc[12]) {
  float sign = 1.f;
  if constexpr (MU == 3) {
    if (g.apt && x3 == (BACK ? 0 : g.L[3] - 1)) sign = -1.f;
  }
  int64_t sy;
  if constexpr (STEP) {
    sy = neighbour(g, s, l, tc, MU, !BACK);
  } else {
    int y[4] = {tc[0] * g.T[0] + l[0], tc[1] * g.T[1] + l[1], tc[2] * g.T[2] + l[2], x3};
    if constexpr (!BACK)
      y[MU] = (y[MU] + 1 == g.L[MU]) ? 0 : y[MU] + 1;
    else
      y[MU] = (y[MU] == 0) ? g.L[MU] - 1 : y[MU] - 1;
    sy = cb_index(g, y);
  }
  unsigned v[12];
  load_chunks16(in.d, sy, v);
  const float scale = in.norm[sy] * sign;
  using PJ = Proj<MU, S>;
  hf2 f0[6], f1[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    hform<PJ::k0, BACK>(hf2_bits(v[a]), hf2_bits(v[3 * PJ::b0 + a]), f0[a], f1[a]);
    hform<PJ::k1, BACK>(hf2_bits(v[3 + a]), hf2_bits(v[3 * PJ::b1 + a]), f0[3 + a], f1[3 + a]);
  }
  // the link: rows 0 and 1 as stored, row 2 = conj(row0 x row1)
  const int lp = BACK ? 1 - p : p;
  const int64_t ls = BACK ? sy : s;
  hf2 u[9];
  {
    unsigned w[6];
    load_link16_raw(gauge, g.nblk, lp, MU, ls, w);
#pragma unroll
    for (int c = 0; c < 6; ++c) u[c] = hf2_bits(w[c]);
  }
  {
    // conj(a b - c d): Re = dot2(a, cj(b)) - dot2(c, cj(d)), -Im = dot2(c, sw(d)) - dot2(a, sw(b))
    auto cj = [](hf2 z) { return hf2{z.x, -z.y}; };
    auto sw = [](hf2 z) { return hf2{z.y, z.x}; };
    auto ng = [](hf2 z) { return hf2{-z.x, -z.y}; };
    auto row2 = [&](hf2 a, hf2 b, hf2 c, hf2 d) {
      const float re = dot2(a, cj(b), dot2(ng(c), cj(d), 0.f));
      const float mi = dot2(c, sw(d), dot2(ng(a), sw(b), 0.f));
      return hf2{(_Float16)re, (_Float16)mi};
    };
    u[6] = row2(u[1], u[5], u[2], u[4]);
    u[7] = row2(u[2], u[3], u[0], u[5]);
    u[8] = row2(u[0], u[4], u[1], u[3]);
  }
  // w = U h (forward) or U^+ h (backward), FP32
  C<float> w[6];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const hf2 ub = BACK ? u[3 * b + a] : u[3 * a + b];
        re = dot2(ub, f0[3 * k + b], re);
        im = dot2(ub, f1[3 * k + b], im);
      }
      w[3 * k + a] = C<float>{scale * re, scale * im};
    }
  reconstruct_add<MU, S>(acc, w);
}

template <int MU, int S, bool BACK, bool STEP, class P>
__device__ __forceinline__ void hop_dir(const Geo& g, const Field<P>& in,
                                        const typename P::S* __restrict__ gauge, int p,
                                        int64_t s, const int l[4], const int tc[4], int x3,
                                        C<typename P::R> acc[12]) {
  using R = typename P::R;
  if constexpr (P::id == LQ_F16 && LQ_HOP16_PACKED) {
    hop_dir16<MU, S, BACK, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
    return;
  }
  R sign = (R)1;
  if constexpr (MU == 3) {
    if (g.apt && x3 == (BACK ? 0 : g.L[3] - 1)) sign = (R)-1;
  }
  // Neighbour number from its coordinates.  (A division-free step,
  // `neighbour()` in site_index.h, gives the same numbers but lets the
  // compiler hoist all eight hops' loads: 256 VGPRs and spills.)
  int y[4] = {tc[0] * g.T[0] + l[0], tc[1] * g.T[1] + l[1], tc[2] * g.T[2] + l[2], x3};
  if constexpr (!BACK)
    y[MU] = (y[MU] + 1 == g.L[MU]) ? 0 : y[MU] + 1;
  else
    y[MU] = (y[MU] == 0) ? g.L[MU] - 1 : y[MU] - 1;
  const int64_t sy = cb_index(g, y);
  C<R> v[12];
  const R scale = load_raw<P>(in, sy, v) * sign;
  C<R> h[6];
  project<MU, S>(v, h);
#pragma unroll
  for (int c = 0; c < 6; ++c) h[c] = scale * h[c];
  C<R> u[9];
  if constexpr (!BACK)
    load_link<P>(gauge, g.nblk, p, MU, s, u);
  else
    load_link<P>(gauge, g.nblk, 1 - p, MU, sy, u);
  C<R> w[6];
  link_mul<BACK>(u, h, w);
  reconstruct_add<MU, S>(acc, w);
}

// acc = (H psi)(x) (DAG: H^dagger) restricted to output site s of parity p.
// STEP, GROUP: the FP16 neighbour numbering (hop_dir16) and the hops per
// scheduling group; the plain hopping kernel takes (true, 8), the fused
// solver kernels the defaults.
template <bool DAG, bool STEP = false, int GROUP = LQ_HOP_GROUP, class P>
__device__ __forceinline__ void hop_site(const Geo& g, const Field<P>& in,
                                         const typename P::S* __restrict__ gauge, int p,
                                         int64_t s, C<typename P::R> acc[12]) {
  using R = typename P::R;
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = C<R>{(R)0, (R)0};
  int l[4], tc[4];
  site_local(g, p, s, l, tc);
  const int x3 = tc[3] * g.T[3] + l[3];
  constexpr int SF = DAG ? -1 : 1;  // forward-hop projector sign
  // The scheduling barriers keep the loads of at most GROUP hops in flight
  // per thread: hoisting all eight (144 loads) would cost registers and with
  // them the occupancy that hides memory latency on this bandwidth-bound
  // kernel.
  hop_dir<0, SF, false, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 2) __builtin_amdgcn_sched_barrier(0);
  hop_dir<0, -SF, true, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 4) __builtin_amdgcn_sched_barrier(0);
  hop_dir<1, SF, false, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 2) __builtin_amdgcn_sched_barrier(0);
  hop_dir<1, -SF, true, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 8) __builtin_amdgcn_sched_barrier(0);
  hop_dir<2, SF, false, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 2) __builtin_amdgcn_sched_barrier(0);
  hop_dir<2, -SF, true, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 4) __builtin_amdgcn_sched_barrier(0);
  hop_dir<3, SF, false, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
  if constexpr (GROUP < 2) __builtin_amdgcn_sched_barrier(0);
  hop_dir<3, -SF, true, STEP>(g, in, gauge, p, s, l, tc, x3, acc);
}

// ---------------------------------------------------------------- clover
// Per site two Hermitian 6x6 blocks (spins {0,1} and {2,3} x colour), each
// stored as 18 complex slots: slots 0..2 hold the real diagonal in pairs
// (d0,d1),(d2,d3),(d4,d5); slots 3..17 the upper triangle row by row.
__host__ __device__ constexpr int tri_idx(int r, int c) {  // r < c
  return r * 5 - r * (r - 1) / 2 + c - r - 1;
}

template <class P>
__device__ __forceinline__ void clover_mul(const typename P::S* __restrict__ cl, int64_t s,
                                           const C<typename P::R> x[12],
                                           C<typename P::R> y[12]) {
  using R = typename P::R;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    C<R> m[18];
    if constexpr (P::id == LQ_F32) {
      const f32x4* q = reinterpret_cast<const f32x4*>(cl);
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const f32x4 w = __builtin_nontemporal_load(q + ((s >> 6) * 18 + 9 * b + j) * SB + (s & 63));
        m[2 * j] = {w.x, w.y};
        m[2 * j + 1] = {w.z, w.w};
      }
    } else if constexpr (P::id == LQ_F16) {
      const unsigned* u = reinterpret_cast<const unsigned*>(cl);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const h16x4 w = __builtin_nontemporal_load(
            reinterpret_cast<const h16x4*>(u + clov16_idx(s, 18 * b + 4 * j)));
        m[4 * j] = h2_to_c(w.x);
        m[4 * j + 1] = h2_to_c(w.y);
        m[4 * j + 2] = h2_to_c(w.z);
        m[4 * j + 3] = h2_to_c(w.w);
      }
      const h16x2 t = __builtin_nontemporal_load(
          reinterpret_cast<const h16x2*>(u + clov16_idx(s, 18 * b + 16)));
      m[16] = h2_to_c(t.x);
      m[17] = h2_to_c(t.y);
    } else {
#pragma unroll
      for (int k = 0; k < 18; ++k) m[k] = ldnt<P>(cl, clov_idx(s, 18 * b + k));
    }
    const C<R>* xb = x + 6 * b;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const R d = (r & 1) ? m[r >> 1].im : m[r >> 1].re;
      C<R> acc = d * xb[r];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        if (c == r) continue;
        if (r < c)
          acc = acc + m[3 + tri_idx(r, c)] * xb[c];
        else
          acc = acc + cmul_conj(m[3 + tri_idx(c, r)], xb[c]);
      }
      y[6 * b + r] = acc;
    }
  }
}

}  // namespace lq
