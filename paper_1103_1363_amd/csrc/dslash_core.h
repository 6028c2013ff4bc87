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
#pragma unroll
  for (int c = 0; c < 6; ++c) u[c] = ldnt<P>(gauge, link_idx(nblk, p, mu, s, c));
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

template <int MU, int S, bool BACK, class P>
__device__ __forceinline__ void hop_dir(const Geo& g, const Field<P>& in,
                                        const typename P::S* __restrict__ gauge, int p,
                                        int64_t s, const int l[4], const int tc[4], int x3,
                                        C<typename P::R> acc[12]) {
  using R = typename P::R;
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
template <bool DAG, class P>
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
  // The scheduling barriers keep the loads of at most two hops in flight per
  // thread: hoisting all eight (144 loads) would cost registers and with them
  // the occupancy that hides memory latency on this bandwidth-bound kernel.
  hop_dir<0, SF, false>(g, in, gauge, p, s, l, tc, x3, acc);
  hop_dir<0, -SF, true>(g, in, gauge, p, s, l, tc, x3, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_dir<1, SF, false>(g, in, gauge, p, s, l, tc, x3, acc);
  hop_dir<1, -SF, true>(g, in, gauge, p, s, l, tc, x3, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_dir<2, SF, false>(g, in, gauge, p, s, l, tc, x3, acc);
  hop_dir<2, -SF, true>(g, in, gauge, p, s, l, tc, x3, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_dir<3, SF, false>(g, in, gauge, p, s, l, tc, x3, acc);
  hop_dir<3, -SF, true>(g, in, gauge, p, s, l, tc, x3, acc);
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
#pragma unroll
    for (int k = 0; k < 18; ++k) m[k] = ldnt<P>(cl, clov_idx(s, 18 * b + k));
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
