// Fused kernels of BiCGStab (van der Vorst) on the Schur operator Mhat,
// with complex scalars kept on the device.
//
// One iteration (r, rh = shadow residual, x in the vector precision;
// p, v, s, tt and the odd temporary t in the operator precision):
//   B1   t  = A_oo^-1 H_oe p                      (cg_k1)
//   B2   v  = A_ee p - kappa^2 H_eo t,    alpha = rho / <rh, v>
//   B3   s  = r - alpha v
//   B4   t  = A_oo^-1 H_oe s                      (cg_k1)
//   B5   tt = A_ee s - kappa^2 H_eo t,    omega = <tt, s> / <tt, tt>
//   B6   x += alpha p + omega s,  r = s - omega tt,
//        rho' = <rh, r>, beta = (rho'/rho)(alpha/omega), stopping tests
//   B7   p  = r + beta (p - omega v)
// The paper names no Krylov method besides CG and FGCR; BiCGStab is the
// textbook recurrence, written from its definition.
#pragma once

#include "solver_kernels.h"

namespace lq {

struct BiState {
  double rho[2], alpha[2], omega[2], beta[2];
  double rr;       // |r|^2 (recurrence)
  double rr_max;   // max |r|^2 since the last reliable update
  double rrh;      // |rh|^2 (for the breakdown test)
  double target2;  // stop when rr <= target2
  double delta2;   // reliable update when rr < delta2 * rr_max (0: never)
  int active;
  int reason;      // as CGState; R_NAN also marks a rho breakdown
  int iter;
  int maxiter;
};

__device__ __forceinline__ C<double> cdiv(C<double> a, C<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

template <class PA, class PB>
__device__ __forceinline__ void site_dot(const C<typename PA::R> a[12],
                                         const C<typename PB::R> b[12], double& re, double& im) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double ar = (double)a[c].re, ai = (double)a[c].im;
    const double br = (double)b[c].re, bi = (double)b[c].im;
    re += ar * br + ai * bi;
    im += ar * bi - ai * br;
  }
}

// B2 / B5: y = A_ee in - kappa^2 H_eo t; MODE 0: partials of <rh, y>;
// MODE 1: partials of <y, in> and <y, y>.
template <class PO, class PV, int MODE>
LQ_HOP_KERNEL(PO) void bi_hop_eo(Geo g, const int* __restrict__ active, Field<PO> y, Field<PO> t,
                                  Field<PO> in, Field<PV> rh,
                                  const typename PO::S* __restrict__ gauge,
                                  const typename PO::S* __restrict__ aee, typename PO::R k2,
                                  RedBuf rb) {
  using R = typename PO::R;
  if (!*active) return;
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * SBLK + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (s < g.vh) {
    C<R> acc[12], iv[12], o[12];
    hop_site<false>(g, t, gauge, 0, s, acc);
    load_scaled<PO>(in, s, iv);
    clover_mul<PO>(aee, s, iv, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = o[c] - k2 * acc[c];
    store_spinor<PO>(y, s, o);
    if constexpr (MODE == 0) {
      C<typename PV::R> h[12];
      load_scaled<PV>(rh, s, h);
      site_dot<PV, PO>(h, o, v[0], v[1]);
    } else {
      site_dot<PO, PO>(o, iv, v[0], v[1]);
      v[2] = site_norm2(o);
    }
  }
  block_partial<3>(v, rb.part);
}

struct FinBiAlpha {
  BiState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;
    const C<double> d = {tot[0], tot[1]};
    const double dn = d.re * d.re + d.im * d.im;
    if (!(dn > 0.0) || !isfinite(dn)) {
      st->reason = R_NAN;
      st->active = 0;
      return;
    }
    const C<double> a = cdiv(C<double>{st->rho[0], st->rho[1]}, d);
    st->alpha[0] = a.re;
    st->alpha[1] = a.im;
  }
};

struct FinBiOmega {
  BiState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;
    const double tt = tot[2];
    if (!(tt > 0.0) || !isfinite(tt)) {
      st->reason = R_NAN;
      st->active = 0;
      return;
    }
    st->omega[0] = tot[0] / tt;
    st->omega[1] = tot[1] / tt;
  }
};

// B3: s = r - alpha v
template <class PO, class PV>
__global__ __launch_bounds__(SBLK) void bi_s(Geo g, const BiState* __restrict__ st, Field<PO> sf,
                                             Field<PV> r, Field<PO> v) {
  using R = typename PO::R;
  if (!st->active) return;
  const int64_t s = (int64_t)blockIdx.x * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  const C<R> al = {(R)st->alpha[0], (R)st->alpha[1]};
  C<R> a[12], b[12];
  load_scaled<PV>(r, s, a);
  load_scaled<PO>(v, s, b);
#pragma unroll
  for (int c = 0; c < 12; ++c) a[c] = a[c] - al * b[c];
  store_spinor<PO>(sf, s, a);
}

// B6: x += alpha p + omega s;  r = s - omega tt;  partials <rh, r>, |r|^2
template <class PO, class PV>
__global__ __launch_bounds__(SBLK) void bi_update(Geo g, const BiState* __restrict__ st,
                                                  Field<PV> x, Field<PV> r, Field<PV> rh,
                                                  Field<PO> p, Field<PO> sf, Field<PO> tt,
                                                  RedBuf rb) {
  using R = typename PO::R;
  if (!st->active) return;
  const int64_t s = (int64_t)blockIdx.x * SBLK + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (s < g.vh) {
    const C<R> al = {(R)st->alpha[0], (R)st->alpha[1]};
    const C<R> om = {(R)st->omega[0], (R)st->omega[1]};
    C<R> a[12], b[12], c2[12];
    load_scaled<PV>(x, s, a);
    load_scaled<PO>(p, s, b);
    load_scaled<PO>(sf, s, c2);
#pragma unroll
    for (int c = 0; c < 12; ++c) a[c] = a[c] + al * b[c] + om * c2[c];
    store_spinor<PV>(x, s, a);
    load_scaled<PO>(tt, s, b);
#pragma unroll
    for (int c = 0; c < 12; ++c) a[c] = c2[c] - om * b[c];
    store_spinor<PV>(r, s, a);
    load_scaled<PV>(rh, s, b);
    site_dot<PV, PV>(b, a, v[0], v[1]);
    v[2] = site_norm2(a);
  }
  block_partial<3>(v, rb.part);
}

struct FinBiRho {
  BiState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;
    const C<double> rho_new = {tot[0], tot[1]};
    const double rr = tot[2];
    st->iter += 1;
    st->rr = rr;
    int reason = R_RUN;
    if (!isfinite(rr) || !isfinite(rho_new.re) || !isfinite(rho_new.im)) {
      reason = R_NAN;
    } else if (rr <= st->target2) {
      reason = R_CONV;
    } else if (st->delta2 > 0.0 && rr < st->delta2 * st->rr_max) {
      reason = R_RELIABLE;
    } else if (sqrt(rho_new.re * rho_new.re + rho_new.im * rho_new.im) <
               1e-30 * sqrt(rr * st->rrh)) {
      reason = R_RELIABLE;  // rho breakdown: restart from the true residual
    } else if (st->iter >= st->maxiter) {
      reason = R_MAXITER;
    }
    if (reason == R_RUN) {
      const C<double> ra = cdiv(rho_new, C<double>{st->rho[0], st->rho[1]});
      const C<double> ao = cdiv(C<double>{st->alpha[0], st->alpha[1]},
                                C<double>{st->omega[0], st->omega[1]});
      const C<double> b = ra * ao;
      st->beta[0] = b.re;
      st->beta[1] = b.im;
      st->rho[0] = rho_new.re;
      st->rho[1] = rho_new.im;
      if (rr > st->rr_max) st->rr_max = rr;
    } else {
      st->reason = reason;
      st->active = 0;
    }
  }
};

// B7: p = r + beta (p - omega v)
template <class PO, class PV>
__global__ __launch_bounds__(SBLK) void bi_p(Geo g, const BiState* __restrict__ st, Field<PO> p,
                                             Field<PV> r, Field<PO> v) {
  using R = typename PO::R;
  if (!st->active) return;
  const int64_t s = (int64_t)blockIdx.x * SBLK + threadIdx.x;
  if (s >= g.vh) return;
  const C<R> be = {(R)st->beta[0], (R)st->beta[1]};
  const C<R> om = {(R)st->omega[0], (R)st->omega[1]};
  C<R> a[12], b[12], c2[12];
  load_scaled<PV>(r, s, a);
  load_scaled<PO>(p, s, b);
  load_scaled<PO>(v, s, c2);
#pragma unroll
  for (int c = 0; c < 12; ++c) b[c] = a[c] + be * (b[c] - om * c2[c]);
  store_spinor<PO>(p, s, b);
}

}  // namespace lq
