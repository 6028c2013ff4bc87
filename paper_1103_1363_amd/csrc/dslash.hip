// Even-odd hopping term, clover application and the Schur operator
//   Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe   (Mhat^+ = A_ee - kappa^2 H^+_eo A_oo^{-1} H^+_oe)
// as stand-alone kernels (one output site per thread).  The solvers use
// fused variants of the same per-site routines (solver.hip).
#include "dslash_core.h"

namespace lq {

namespace {

constexpr int BLK = 256;

template <class P, bool DAG>
LQ_HOP_KERNEL(P) void dslash_kernel(Geo g, int p, Field<P> out, Field<P> in,
                                                     const typename P::S* __restrict__ gauge) {
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * BLK + threadIdx.x;
  if (s >= g.vh) return;
  C<typename P::R> acc[12];
  // FP16: the division-free neighbour step and no scheduling barriers
  // (measured fastest for this kernel alone); FP64/FP32: the defaults
  constexpr bool h16 = P::id == LQ_F16;
  hop_site<DAG, h16, h16 ? 8 : LQ_HOP_GROUP>(g, in, gauge, p, s, acc);
  store_spinor<P>(out, s, acc);
}

template <class P>
__global__ __launch_bounds__(BLK) void clover_kernel(Geo g, Field<P> out, Field<P> in,
                                                     const typename P::S* __restrict__ cl) {
  const int64_t s = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (s >= g.vh) return;
  C<typename P::R> x[12], y[12];
  const typename P::R n = load_raw<P>(in, s, x);
#pragma unroll
  for (int c = 0; c < 12; ++c) x[c] = n * x[c];
  clover_mul<P>(cl, s, x, y);
  store_spinor<P>(out, s, y);
}

// t_o = A_oo^{-1} H_oe in_e   (DAG: H^+ blocks)
template <class P, bool DAG>
LQ_HOP_KERNEL(P) void schur_k1_kernel(Geo g, Field<P> out, Field<P> in,
                                                       const typename P::S* __restrict__ gauge,
                                                       const typename P::S* __restrict__ ainv) {
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * BLK + threadIdx.x;
  if (s >= g.vh) return;
  C<typename P::R> acc[12], y[12];
  hop_site<DAG>(g, in, gauge, 1, s, acc);
  clover_mul<P>(ainv, s, acc, y);
  store_spinor<P>(out, s, y);
}

// out_e = A_ee x_e - kappa^2 H_eo t_o
template <class P, bool DAG>
LQ_HOP_KERNEL(P) void schur_k2_kernel(Geo g, Field<P> out, Field<P> t,
                                                       Field<P> x,
                                                       const typename P::S* __restrict__ gauge,
                                                       const typename P::S* __restrict__ aee,
                                                       typename P::R k2) {
  using R = typename P::R;
  const int64_t s = xcd_block(blockIdx.x, gridDim.x) * BLK + threadIdx.x;
  if (s >= g.vh) return;
  C<R> acc[12], xv[12], y[12];
  hop_site<DAG>(g, t, gauge, 0, s, acc);
  const R n = load_raw<P>(x, s, xv);
#pragma unroll
  for (int c = 0; c < 12; ++c) xv[c] = n * xv[c];
  clover_mul<P>(aee, s, xv, y);
#pragma unroll
  for (int c = 0; c < 12; ++c) y[c] = y[c] - k2 * acc[c];
  store_spinor<P>(out, s, y);
}

template <class P>
void dslash_t(lq_ctx* ctx, void* out, const void* in, int p, int dag) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * dslash_site_bytes(P::id);
  Field<P> fo = field_at<P>(out, g.nblk);
  Field<P> fi = field_at<P>(const_cast<void*>(in), g.nblk);
  auto* gp = reinterpret_cast<const typename P::S*>(ctx->gauge[P::id]);
  dim3 grid(grid_for(g.vh, BLK));
  if (dag)
    hipLaunchKernelGGL((dslash_kernel<P, true>), grid, dim3(BLK), 0, ctx->cur, g, p, fo, fi,
                       gp);
  else
    hipLaunchKernelGGL((dslash_kernel<P, false>), grid, dim3(BLK), 0, ctx->cur, g, p, fo, fi,
                       gp);
  LQ_HIP(hipGetLastError());
}

template <class P>
void clover_t(lq_ctx* ctx, void* out, const void* in, const void* cl) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * (clover_site_bytes(P::id) + 2 * spinor_site_bytes(P::id));
  Field<P> fo = field_at<P>(out, g.nblk);
  Field<P> fi = field_at<P>(const_cast<void*>(in), g.nblk);
  hipLaunchKernelGGL(clover_kernel<P>, dim3(grid_for(g.vh, BLK)), dim3(BLK), 0, ctx->cur, g,
                     fo, fi, reinterpret_cast<const typename P::S*>(cl));
  LQ_HIP(hipGetLastError());
}

template <class P, bool DAG>
void schur_t(lq_ctx* ctx, void* out, const void* in, void* tmp) {
  const Geo& g = ctx->geo;
  // K1: links, input, clover, output; K2: links, t, x, clover, output
  ctx->bytes += (double)g.vh * (16 * link_site_bytes(P::id) + 5 * spinor_site_bytes(P::id) +
                                2 * clover_site_bytes(P::id));
  Field<P> fo = field_at<P>(out, g.nblk);
  Field<P> fi = field_at<P>(const_cast<void*>(in), g.nblk);
  Field<P> ft = field_at<P>(tmp, g.nblk);
  auto* gp = reinterpret_cast<const typename P::S*>(ctx->gauge[P::id]);
  auto* ai = reinterpret_cast<const typename P::S*>(ctx->clov.ainv_oo[P::id]);
  auto* ae = reinterpret_cast<const typename P::S*>(ctx->clov.a_ee[P::id]);
  dim3 grid(grid_for(g.vh, BLK));
  hipLaunchKernelGGL((schur_k1_kernel<P, DAG>), grid, dim3(BLK), 0, ctx->cur, g, ft, fi, gp,
                     ai);
  LQ_HIP(hipGetLastError());
  const typename P::R k2 = (typename P::R)(ctx->clov.kappa * ctx->clov.kappa);
  hipLaunchKernelGGL((schur_k2_kernel<P, DAG>), grid, dim3(BLK), 0, ctx->cur, g, fo, ft, fi,
                     gp, ae, k2);
  LQ_HIP(hipGetLastError());
}

}  // namespace

void dslash(lq_ctx* ctx, void* out, const void* in, int out_parity, int dagger, int prec) {
  switch (prec) {
    case LQ_F64: dslash_t<P64>(ctx, out, in, out_parity, dagger); break;
    case LQ_F32: dslash_t<P32>(ctx, out, in, out_parity, dagger); break;
    default: dslash_t<P16>(ctx, out, in, out_parity, dagger); break;
  }
}

void clover_apply(lq_ctx* ctx, void* out, const void* in, int parity, int inverse, int prec) {
  const Clover& c = ctx->clov;
  const void* cl = nullptr;
  if (prec == LQ_F64) {
    cl = inverse ? c.ainv64[parity] : c.a64[parity];
  } else {
    LQ_CHECK((parity == LQ_EVEN && !inverse) || (parity == LQ_ODD && inverse), LQ_EINVAL,
             "FP32/FP16 clover fields exist for A_ee and A_oo^-1 only");
    cl = inverse ? c.ainv_oo[prec] : c.a_ee[prec];
  }
  switch (prec) {
    case LQ_F64: clover_t<P64>(ctx, out, in, cl); break;
    case LQ_F32: clover_t<P32>(ctx, out, in, cl); break;
    default: clover_t<P16>(ctx, out, in, cl); break;
  }
}

void schur(lq_ctx* ctx, void* out, const void* in, void* tmp, int dagger, int prec) {
  switch (prec * 2 + (dagger ? 1 : 0)) {
    case 0: schur_t<P64, false>(ctx, out, in, tmp); break;
    case 1: schur_t<P64, true>(ctx, out, in, tmp); break;
    case 2: schur_t<P32, false>(ctx, out, in, tmp); break;
    case 3: schur_t<P32, true>(ctx, out, in, tmp); break;
    case 4: schur_t<P16, false>(ctx, out, in, tmp); break;
    default: schur_t<P16, true>(ctx, out, in, tmp); break;
  }
}

}  // namespace lq
