// Gauge-field upload with 12-real compression, and spinor packing between
// the host canonical layout and the device site-blocked layouts.
#include "lq_internal.h"

namespace lq {

namespace {

// One thread per (site, direction): writes rows 0 and 1 of U_mu(x) in FP64,
// FP32 and FP16 to the compressed arrays of the site's parity and reports
// max(|U U^dagger - 1|, |det U - 1|) for the block.
__global__ void compress_gauge_kernel(Geo g, const double2* __restrict__ host, double2* g64,
                                      float2* g32, __half2* g16, double* blockmax,
                                      int64_t nlinks) {
  __shared__ double red[256];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double err = 0.0;
  if (t < nlinks) {
    int64_t i = t >> 2;
    int mu = (int)(t & 3);
    int x[4];
    canonical_coords(g, i, x);
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int64_t s = cb_index(g, x);
    C<double> u[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double2 v = host[t * 9 + a * 3 + b];
        u[a][b] = {v.x, v.y};
      }
    // unitarity
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        C<double> acc = {0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 3; ++c) acc = acc + u[a][c] * conj(u[b][c]);
        if (a == b) acc.re -= 1.0;
        err = fmax(err, sqrt(norm2(acc)));
      }
    C<double> det = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[2][1]) -
                    u[0][1] * (u[1][0] * u[2][2] - u[1][2] * u[2][0]) +
                    u[0][2] * (u[1][0] * u[2][1] - u[1][1] * u[2][0]);
    det.re -= 1.0;
    err = fmax(err, sqrt(norm2(det)));
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      C<double> v = u[c / 3][c % 3];
      int64_t k = link_idx(g.nblk, p, mu, s, c);
      g64[k] = make_double2(v.re, v.im);
      g32[link32_idx(g.nblk, p, mu, s, c)] = make_float2((float)v.re, (float)v.im);
      _Float16 hr = (_Float16)v.re, hi = (_Float16)v.im;
      __half2 h;
      h.x = __half(hr);
      h.y = __half(hi);
      g16[link16_idx(g.nblk, p, mu, s, c)] = h;
    }
  }
  red[threadIdx.x] = err;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

// Device site of host index t and its parity.  parity EVEN/ODD: t ranks
// the site among the sites of that parity in canonical order (t = i / 2);
// FULL: t is the canonical index i.
__device__ inline int64_t host_to_device_site(const Geo& g, int parity, int64_t t, int& p) {
  int x[4];
  if (parity == LQ_FULL) {
    canonical_coords(g, t, x);
    p = (x[0] + x[1] + x[2] + x[3]) & 1;
  } else {
    canonical_coords(g, 2 * t, x);  // x0 even; the parity picks x0 or x0 + 1
    p = parity;
    x[0] += (p + x[0] + x[1] + x[2] + x[3]) & 1;
  }
  return cb_index(g, x);
}

// Host canonical half or full field (double2 per complex) -> device field.
template <class P>
__global__ void pack_kernel(Geo g, Field<P> f_even, Field<P> f_odd, const double2* __restrict__ src,
                            int64_t n, int parity) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int p = 0;
  const int64_t s = host_to_device_site(g, parity, t, p);
  const Field<P> f = p ? f_odd : f_even;
  double2 v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = src[t * 12 + c];
  if constexpr (P::has_norm) {
    double m = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmax(m, fmax(fabs(v[c].x), fabs(v[c].y)));
    f.norm[s] = (float)m;
    double inv = m > 0.0 ? 1.0 / m : 0.0;
    unsigned u[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      __half2 h;
      h.x = __half((_Float16)(v[c].x * inv));
      h.y = __half((_Float16)(v[c].y * inv));
      __builtin_memcpy(&u[c], &h, 4);
    }
    store_chunks16(f.d, s, u);
  } else {
    C<typename P::R> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = C<typename P::R>{(typename P::R)v[c].x, (typename P::R)v[c].y};
    store_spinor<P>(f, s, w);
  }
}

template <class P>
__global__ void unpack_kernel(Geo g, Field<P> f_even, Field<P> f_odd, double2* __restrict__ dst,
                              int64_t n, int parity) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int p = 0;
  const int64_t s = host_to_device_site(g, parity, t, p);
  const Field<P> f = p ? f_odd : f_even;
  // the stored value is component * scale; form the product in FP64 so the
  // host sees exactly what the field represents
  C<typename P::R> v[12];
  const double sc = (double)load_raw<P>(f, s, v);
#pragma unroll
  for (int c = 0; c < 12; ++c)
    dst[t * 12 + c] = make_double2(sc * (double)v[c].re, sc * (double)v[c].im);
}

// For a half field, dev is that parity's field (both f_even and f_odd
// point at it); for FULL, dev holds the even half then the odd half.
template <class P>
void pack_t(lq_ctx* ctx, void* dev, const double2* src, int parity) {
  const Geo& g = ctx->geo;
  char* base = reinterpret_cast<char*>(dev);
  Field<P> fe = field_at<P>(base, g.nblk);
  Field<P> fo = parity == LQ_FULL ? field_at<P>(base + parity_field_bytes(g.nblk, P::id), g.nblk)
                                  : fe;
  const int64_t n = parity == LQ_FULL ? ctx->V : g.vh;
  ctx->bytes += (double)n * (192.0 + spinor_site_bytes(P::id));
  hipLaunchKernelGGL(pack_kernel<P>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur, g, fe, fo,
                     src, n, parity);
  LQ_HIP(hipGetLastError());
}

template <class P>
void unpack_t(lq_ctx* ctx, double2* dst, const void* dev, int parity) {
  const Geo& g = ctx->geo;
  char* base = reinterpret_cast<char*>(const_cast<void*>(dev));
  Field<P> fe = field_at<P>(base, g.nblk);
  Field<P> fo = parity == LQ_FULL ? field_at<P>(base + parity_field_bytes(g.nblk, P::id), g.nblk)
                                  : fe;
  const int64_t n = parity == LQ_FULL ? ctx->V : g.vh;
  ctx->bytes += (double)n * (192.0 + spinor_site_bytes(P::id));
  hipLaunchKernelGGL(unpack_kernel<P>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur, g, fe,
                     fo, dst, n, parity);
  LQ_HIP(hipGetLastError());
}

}  // namespace

namespace {

// unit links U_mu(x) = 1 in the host layout (the tile tuner's operator: the
// kernels' work does not depend on the link values)
__global__ void unit_links_kernel(double2* __restrict__ u, int64_t nlinks) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlinks) return;
#pragma unroll
  for (int k = 0; k < 9; ++k) u[t * 9 + k] = make_double2(k % 4 == 0 ? 1.0 : 0.0, 0.0);
}

void compress_staged_gauge(lq_ctx* ctx, const double2* st);

}  // namespace

void upload_gauge(lq_ctx* ctx, const double* host_U) {
  const int64_t nlinks = ctx->V * 4;
  const size_t host_bytes = (size_t)nlinks * 9 * 16;
  double2* st = reinterpret_cast<double2*>(staging(ctx, host_bytes));
  LQ_HIP(hipMemcpyAsync(st, host_U, host_bytes, hipMemcpyHostToDevice, ctx->cur));
  compress_staged_gauge(ctx, st);
}

void upload_unit_gauge(lq_ctx* ctx) {
  const int64_t nlinks = ctx->V * 4;
  double2* st = reinterpret_cast<double2*>(staging(ctx, (size_t)nlinks * 9 * 16));
  hipLaunchKernelGGL(unit_links_kernel, dim3(grid_for(nlinks, 256)), dim3(256), 0, ctx->cur, st,
                     nlinks);
  LQ_HIP(hipGetLastError());
  compress_staged_gauge(ctx, st);
}

namespace {

void compress_staged_gauge(lq_ctx* ctx, const double2* st) {
  const Geo& g = ctx->geo;
  const int64_t nlinks = ctx->V * 4;
  const int64_t ncomp = 2 * 4 * g.nblk * 6 * SB;
  for (int p = 0; p < 3; ++p) {
    if (!ctx->gauge[p]) {
      size_t b = (size_t)ncomp * (p == 0 ? 16 : p == 1 ? 8 : 4);
      LQ_HIP(hipMalloc(&ctx->gauge[p], b));
      LQ_HIP(hipMemsetAsync(ctx->gauge[p], 0, b, ctx->cur));
    }
  }
  const int nb = grid_for(nlinks, 256);
  double* bm = nullptr;
  LQ_HIP(hipMalloc(&bm, sizeof(double) * nb));
  hipLaunchKernelGGL(compress_gauge_kernel, dim3(nb), dim3(256), 0, ctx->cur, g, st,
                     (double2*)ctx->gauge[0], (float2*)ctx->gauge[1], (__half2*)ctx->gauge[2], bm,
                     nlinks);
  hipError_t le = hipGetLastError();
  std::vector<double> hbm(nb);
  hipError_t ce = hipMemcpyAsync(hbm.data(), bm, sizeof(double) * nb, hipMemcpyDeviceToHost,
                                 ctx->cur);
  hipError_t se = hipStreamSynchronize(ctx->cur);
  (void)hipFree(bm);
  LQ_HIP(le);
  LQ_HIP(ce);
  LQ_HIP(se);
  double worst = 0.0;
  for (double v : hbm) worst = v > worst ? v : worst;
  if (!(worst <= 1e-12)) {
    ctx->have_gauge = false;
    throw Error(LQ_EINVAL, "gauge field is not SU(3): max(|UU^+ - 1|, |det U - 1|) = " +
                               std::to_string(worst));
  }
  ctx->have_gauge = true;
  ctx->clov.valid = false;
  ctx->mr_links_ok = ctx->mr_clov_ok = false;
}

}  // namespace

void pack_spinor(lq_ctx* ctx, void* dev, const double2* src, int prec, int parity) {
  switch (prec) {
    case LQ_F64: pack_t<P64>(ctx, dev, src, parity); break;
    case LQ_F32: pack_t<P32>(ctx, dev, src, parity); break;
    default: pack_t<P16>(ctx, dev, src, parity); break;
  }
}

void unpack_spinor(lq_ctx* ctx, double2* dst, const void* dev, int prec, int parity) {
  switch (prec) {
    case LQ_F64: unpack_t<P64>(ctx, dst, dev, parity); break;
    case LQ_F32: unpack_t<P32>(ctx, dst, dev, parity); break;
    default: unpack_t<P16>(ctx, dst, dev, parity); break;
  }
}

}  // namespace lq
