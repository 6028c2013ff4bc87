// Fused kernels of the CG iteration on the normal equations of the Schur
// operator, Mhat^+ Mhat x = Mhat^+ bhat, with the scalars kept on the device.
//
// One iteration (p, q, t, x, r, rt are device fields; r is the normal
// residual Mhat^+ (bhat - Mhat x), rt the Schur residual bhat - Mhat x
// carried by recurrence so that the stopping test uses the true residual):
//   K1   t  = A_oo^-1 H_oe p
//   K2   q  = A_ee p - kappa^2 H_eo t,            alpha = |r|^2 / |q|^2
//   K1+  t  = A_oo^-1 H^+_oe q
//   K4   s  = A_ee q - kappa^2 H^+_eo t  (not stored),
//        x += alpha p,  r -= alpha s,  rt -= alpha q,
//        beta = |r_new|^2 / |r|^2, convergence / reliable-update tests
//   K5   p  = r + beta p
// K2 and K4 write per-workgroup partial sums; a one-workgroup kernel after
// each forms the totals and the scalars (reduce.h).
// Every kernel returns at once when the device flag `active` is 0, so a
// captured graph of several iterations can be replayed past the point where
// the solver stopped.
#pragma once

#include "dslash_core.h"
#include "reduce.h"

namespace lq {

struct CGState {
  double rr;       // |r|^2, normal residual (inner precision)
  double alpha, beta;
  double qq;
  double rt2;      // |rt|^2, Schur residual recurrence
  double rt2_max;  // max |rt|^2 since the last reliable update
  double target2;  // stop when rt2 <= target2
  double delta2;   // reliable update when rt2 < delta2 * rt2_max (0: never)
  int active;
  int reason;      // 0 running, 1 converged, 2 reliable update due, 3 NaN/breakdown, 4 maxiter
  int iter;
  int maxiter;
};
enum { R_RUN = 0, R_CONV = 1, R_RELIABLE = 2, R_NAN = 3, R_MAXITER = 4 };

constexpr int SBLK = 256;

template <class P>
__device__ __forceinline__ void load_scaled(const Field<P>& f, int64_t s, C<typename P::R> v[12]) {
  const typename P::R n = load_raw<P>(f, s, v);
  if constexpr (P::has_norm) {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = n * v[c];
  }
}

template <class R>
__device__ __forceinline__ double site_norm2(const C<R> v[12]) {
  double a = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double re = (double)v[c].re, im = (double)v[c].im;
    a += re * re + im * im;
  }
  return a;
}

// ---------------------------------------------------------------- site bodies
// The per-site work of each stage, shared by the single-lattice kernels below
// and by the uneven-batch kernels (ensemble.hip), which only differ in how a
// workgroup finds its lattice and its sites.

// t = A_oo^-1 H_oe in (DAG: A_oo^-1 H^+_oe in) at odd site s.
template <class PO, bool DAG>
__device__ __forceinline__ void k1_site(const Geo& g, int64_t s, const Field<PO>& t,
                                        const Field<PO>& in,
                                        const typename PO::S* __restrict__ gauge,
                                        const typename PO::S* __restrict__ ainv) {
  C<typename PO::R> acc[12], y[12];
  hop_site<DAG>(g, in, gauge, 1, s, acc);
  clover_mul<PO>(ainv, s, acc, y);
  store_spinor<PO>(t, s, y);
}

// y = A_ee in - k2 H_eo t (DAG: H^+_eo) at even site s: the Schur operator
// (or its adjoint) once t holds the K1 result; inv receives in(s).
template <class PO, bool DAG>
__device__ __forceinline__ void schur_site(const Geo& g, int64_t s, const Field<PO>& in,
                                           const Field<PO>& t,
                                           const typename PO::S* __restrict__ gauge,
                                           const typename PO::S* __restrict__ aee,
                                           typename PO::R k2, C<typename PO::R> inv[12],
                                           C<typename PO::R> y[12]) {
  C<typename PO::R> acc[12];
  hop_site<DAG>(g, t, gauge, 0, s, acc);
  load_scaled<PO>(in, s, inv);
  clover_mul<PO>(aee, s, inv, y);
#pragma unroll
  for (int c = 0; c < 12; ++c) y[c] = y[c] - k2 * acc[c];
}

// x += alpha p, r -= alpha y, rt -= alpha qv at even site s;
// v = (|r_new|^2, |rt_new|^2) of the site.
template <class PO, class PV>
__device__ __forceinline__ void k4_update_site(int64_t s, typename PO::R alpha,
                                               const Field<PO>& p, const Field<PV>& x,
                                               const Field<PV>& r, const Field<PV>& rt,
                                               const C<typename PO::R> y[12],
                                               const C<typename PO::R> qv[12], double v[2]) {
  using R = typename PO::R;
  static_assert(sizeof(R) == sizeof(typename PV::R), "operator and vector arithmetic differ");
  C<R> a[12], b[12];
  load_scaled<PV>(x, s, a);
  load_scaled<PO>(p, s, b);
#pragma unroll
  for (int c = 0; c < 12; ++c) a[c] = a[c] + alpha * b[c];
  store_spinor<PV>(x, s, a);
  load_scaled<PV>(r, s, a);
#pragma unroll
  for (int c = 0; c < 12; ++c) a[c] = a[c] - alpha * y[c];
  store_spinor<PV>(r, s, a);
  v[0] = site_norm2(a);
  load_scaled<PV>(rt, s, a);
#pragma unroll
  for (int c = 0; c < 12; ++c) a[c] = a[c] - alpha * qv[c];
  store_spinor<PV>(rt, s, a);
  v[1] = site_norm2(a);
}

// p = r + beta p at site s (beta == 0: p = r without reading p).
template <class PO, class PV>
__device__ __forceinline__ void k5_site(int64_t s, typename PO::R beta, const Field<PO>& p,
                                        const Field<PV>& r) {
  using R = typename PO::R;
  C<R> a[12], b[12];
  load_scaled<PV>(r, s, a);
  if (beta != (R)0) {
    load_scaled<PO>(p, s, b);
#pragma unroll
    for (int c = 0; c < 12; ++c) a[c] = a[c] + beta * b[c];
  }
  store_spinor<PO>(p, s, a);
}

// ---------------------------------------------------------------- kernels
template <class PO, bool DAG>
LQ_HOP_KERNEL(PO) void cg_k1(Geo g, const int* __restrict__ active, Field<PO> t,
                                              Field<PO> in, const typename PO::S* __restrict__ gauge,
                                              const typename PO::S* __restrict__ ainv) {
  if (!*active) return;
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  k1_site<PO, DAG>(g, s, t, in, gauge, ainv);
}

struct FinAlpha {
  CGState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;  // the producing kernel did not run
    const double qq = tot[0];
    st->qq = qq;
    if (!(qq > 0.0) || !isfinite(qq)) {
      st->reason = R_NAN;
      st->active = 0;
    } else {
      st->alpha = st->rr / qq;
    }
  }
};

template <class PO>
LQ_HOP_KERNEL(PO) void cg_k2(Geo g, CGState* st, Field<PO> q, Field<PO> t,
                                              Field<PO> p, const typename PO::S* __restrict__ gauge,
                                              const typename PO::S* __restrict__ aee,
                                              typename PO::R k2, RedBuf rb) {
  using R = typename PO::R;
  if (!st->active) return;
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * SBLK + threadIdx.x;
  double v[1] = {0.0};
  if (s < g.vh) {
    C<R> pv[12], y[12];
    schur_site<PO, false>(g, s, p, t, gauge, aee, k2, pv, y);
    store_spinor<PO>(q, s, y);
    v[0] = site_norm2(y);
  }
  block_partial<1>(v, rb.part);
}

struct FinBeta {
  CGState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;  // the producing kernel did not run
    const double rr = tot[0], rt2 = tot[1];
    st->iter += 1;
    st->rt2 = rt2;
    int reason = R_RUN;
    if (!isfinite(rr) || !isfinite(rt2) || !(st->rr > 0.0)) {
      reason = R_NAN;
    } else {
      st->beta = rr / st->rr;
      st->rr = rr;
      if (rt2 <= st->target2)
        reason = R_CONV;
      else if (st->delta2 > 0.0 && rt2 < st->delta2 * st->rt2_max)
        reason = R_RELIABLE;
      else if (st->iter >= st->maxiter)
        reason = R_MAXITER;
      if (rt2 > st->rt2_max) st->rt2_max = rt2;
    }
    if (reason != R_RUN) {
      st->reason = reason;
      st->active = 0;
    }
  }
};

template <class PO, class PV>
LQ_HOP_KERNEL(PO) void cg_k4(Geo g, CGState* st, Field<PO> t, Field<PO> q,
                                              Field<PO> p, Field<PV> x, Field<PV> r, Field<PV> rt,
                                              const typename PO::S* __restrict__ gauge,
                                              const typename PO::S* __restrict__ aee,
                                              typename PO::R k2, RedBuf rb) {
  using R = typename PO::R;
  if (!st->active) return;
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * SBLK + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (s < g.vh) {
    C<R> qv[12], y[12];
    schur_site<PO, true>(g, s, q, t, gauge, aee, k2, qv, y);  // y = Mhat^+ q
    k4_update_site<PO, PV>(s, (R)st->alpha, p, x, r, rt, y, qv, v);
  }
  block_partial<2>(v, rb.part);
}

template <class PO, class PV>
__global__ __launch_bounds__(SBLK) void cg_k5(Geo g, const CGState* __restrict__ st, Field<PO> p,
                                              Field<PV> r) {
  if (!st->active) return;
  const int64_t s = (int64_t)blockIdx.x * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  k5_site<PO, PV>(s, (typename PO::R)st->beta, p, r);
}

// out = a * x + b * y (real coefficients), any precisions; out may alias x or y.
template <class PX, class PY, class PO>
__global__ __launch_bounds__(SBLK) void axpby_kernel(Geo g, Field<PO> out, double a, Field<PX> x,
                                                     double b, Field<PY> y) {
  const int64_t s = (int64_t)blockIdx.x * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  C<typename PX::R> xv[12];
  C<typename PY::R> yv[12];
  load_scaled<PX>(x, s, xv);
  load_scaled<PY>(y, s, yv);
  C<typename PO::R> o[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double re = a * (double)xv[c].re + b * (double)yv[c].re;
    const double im = a * (double)xv[c].im + b * (double)yv[c].im;
    o[c] = C<typename PO::R>{(typename PO::R)re, (typename PO::R)im};
  }
  store_spinor<PO>(out, s, o);
}

template <class PO>
__global__ __launch_bounds__(SBLK) void zero_kernel(Geo g, Field<PO> out) {
  const int64_t s = (int64_t)blockIdx.x * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  C<typename PO::R> o[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) o[c] = C<typename PO::R>{0, 0};
  store_spinor<PO>(out, s, o);
}

}  // namespace lq
