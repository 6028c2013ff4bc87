// Global norm and inner product of device spinor fields (FP64 accumulation).
#include "reduce.h"

namespace lq {

namespace {

constexpr int RBLK = 256;

inline int red_grid(int64_t vh) {
  int g = grid_for(vh, RBLK);
  return g > 2048 ? 2048 : g;
}

template <class P>
__global__ __launch_bounds__(RBLK) void norm2_kernel(Geo g, Field<P> a, RedBuf rb) {
  double v[1] = {0.0};
  for (int64_t s = (int64_t)blockIdx.x * RBLK + threadIdx.x; s < g.vh;
       s += (int64_t)gridDim.x * RBLK) {
    C<typename P::R> x[12];
    const double n = (double)load_raw<P>(a, s, x);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double re = (double)x[c].re, im = (double)x[c].im;
      acc += re * re + im * im;
    }
    v[0] += acc * n * n;
  }
  block_partial<1>(v, rb.part);
}

template <class P>
__global__ __launch_bounds__(RBLK) void dot_kernel(Geo g, Field<P> a, Field<P> b, RedBuf rb) {
  double v[2] = {0.0, 0.0};
  for (int64_t s = (int64_t)blockIdx.x * RBLK + threadIdx.x; s < g.vh;
       s += (int64_t)gridDim.x * RBLK) {
    C<typename P::R> x[12], y[12];
    const double na = (double)load_raw<P>(a, s, x);
    const double nb = (double)load_raw<P>(b, s, y);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const C<double> xd = {(double)x[c].re, (double)x[c].im};
      const C<double> yd = {(double)y[c].re, (double)y[c].im};
      const C<double> z = cmul_conj(xd, yd);
      re += z.re;
      im += z.im;
    }
    v[0] += re * na * nb;
    v[1] += im * na * nb;
  }
  block_partial<2>(v, rb.part);
}

template <class P>
void norm2_t(lq_ctx* ctx, double* out, const void* a) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * spinor_site_bytes(P::id);
  RedBuf rb = red_buf(ctx);
  const int nb = red_grid(g.vh);
  hipLaunchKernelGGL(norm2_kernel<P>, dim3(nb), dim3(RBLK), 0, ctx->cur, g,
                     field_at<P>(const_cast<void*>(a), g.nblk), rb);
  hipLaunchKernelGGL((finalize_kernel<1, NoFin>), dim3(1), dim3(256), 0, ctx->cur, rb, nb,
                     NoFin{});
  LQ_HIP(hipGetLastError());
  LQ_HIP(hipMemcpyAsync(out, rb.result, sizeof(double), hipMemcpyDeviceToHost, ctx->cur));
  LQ_HIP(hipStreamSynchronize(ctx->cur));
}

template <class P>
void dot_t(lq_ctx* ctx, double* out, const void* a, const void* b) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * 2 * spinor_site_bytes(P::id);
  RedBuf rb = red_buf(ctx);
  const int nb = red_grid(g.vh);
  hipLaunchKernelGGL(dot_kernel<P>, dim3(nb), dim3(RBLK), 0, ctx->cur, g,
                     field_at<P>(const_cast<void*>(a), g.nblk),
                     field_at<P>(const_cast<void*>(b), g.nblk), rb);
  hipLaunchKernelGGL((finalize_kernel<2, NoFin>), dim3(1), dim3(256), 0, ctx->cur, rb, nb,
                     NoFin{});
  LQ_HIP(hipGetLastError());
  LQ_HIP(hipMemcpyAsync(out, rb.result, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->cur));
  LQ_HIP(hipStreamSynchronize(ctx->cur));
}

}  // namespace

void norm2(lq_ctx* ctx, double* out, const void* a, int prec) {
  switch (prec) {
    case LQ_F64: norm2_t<P64>(ctx, out, a); break;
    case LQ_F32: norm2_t<P32>(ctx, out, a); break;
    default: norm2_t<P16>(ctx, out, a); break;
  }
}

void dot(lq_ctx* ctx, double* out, const void* a, const void* b, int prec) {
  switch (prec) {
    case LQ_F64: dot_t<P64>(ctx, out, a, b); break;
    case LQ_F32: dot_t<P32>(ctx, out, a, b); break;
    default: dot_t<P16>(ctx, out, a, b); break;
  }
}

}  // namespace lq

namespace {

// Streaming copy, 16 bytes per lane and four per thread in flight: the
// achievable-bandwidth reference of the roofline figures.
constexpr int CPY_BLK = 256, CPY_U = 4;
__global__ __launch_bounds__(CPY_BLK) void stream_copy_kernel(uint4* __restrict__ dst,
                                                              const uint4* __restrict__ src,
                                                              int64_t n) {
  const int64_t i0 = (int64_t)blockIdx.x * CPY_BLK * CPY_U + threadIdx.x;
  uint4 v[CPY_U];
#pragma unroll
  for (int k = 0; k < CPY_U; ++k)
    if (i0 + k * CPY_BLK < n) v[k] = src[i0 + k * CPY_BLK];
#pragma unroll
  for (int k = 0; k < CPY_U; ++k)
    if (i0 + k * CPY_BLK < n) dst[i0 + k * CPY_BLK] = v[k];
}

}  // namespace

extern "C" lq_status lq_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return LQ_EINVAL;
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return LQ_OK;
  const int64_t per = (int64_t)CPY_BLK * CPY_U;
  const int64_t grid = (n + per - 1) / per;
  if (grid > 0x7fffffff) return LQ_EINVAL;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)grid), dim3(CPY_BLK), 0,
                     reinterpret_cast<hipStream_t>(stream), reinterpret_cast<uint4*>(dst),
                     reinterpret_cast<const uint4*>(src), n);
  return hipGetLastError() == hipSuccess ? LQ_OK : LQ_EHIP;
}
