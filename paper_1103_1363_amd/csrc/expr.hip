// C entry points of fused lattice expressions (lattice_expr.h): the SU(3)
// array product of the paper's worked example (section 3, eq. su3vecmul),
// its adjoint forms, a three-factor product that one fused kernel evaluates
// in one pass, and the colour matrix acting on the spinors of a field.
#include <cstring>
#include <vector>

#include "lattice_expr.h"

namespace {

using namespace lq;
using namespace lq::expr;

template <class R>
using MatF = expr::Field<Mat<R>, R>;
template <class R>
using SpinF = expr::Field<Spin<R>, R>;

template <class F>
lq_status guard(F&& f) {
  try {
    f();
    return LQ_OK;
  } catch (const lq::Error& e) {
    return e.code;
  } catch (...) {
    return LQ_EINVAL;
  }
}

bool prec_ok(int prec) { return prec == LQ_F64 || prec == LQ_F32; }

template <class R>
void su3_mul_t(void* u, const void* v, const void* w, const void* x, int64_t n, int form,
               hipStream_t st) {
  MatF<R> U{reinterpret_cast<typename MatF<R>::S*>(u)};
  MatF<R> V{reinterpret_cast<typename MatF<R>::S*>(const_cast<void*>(v))};
  MatF<R> W{reinterpret_cast<typename MatF<R>::S*>(const_cast<void*>(w))};
  switch (form) {
    case LQ_SU3_VW: evaluate(U, V * W, n, st); break;
    case LQ_SU3_VWDAG: evaluate(U, V * adj(W), n, st); break;
    case LQ_SU3_VDAGW: evaluate(U, adj(V) * W, n, st); break;
    default: {
      MatF<R> X{reinterpret_cast<typename MatF<R>::S*>(const_cast<void*>(x))};
      evaluate(U, V * W * X, n, st);
    }
  }
}

template <class R>
void su3_spinor_t(void* out, const void* u, const void* in, int64_t n, int adjoint_u,
                  hipStream_t st) {
  SpinF<R> O{reinterpret_cast<typename SpinF<R>::S*>(out)};
  SpinF<R> I{reinterpret_cast<typename SpinF<R>::S*>(const_cast<void*>(in))};
  MatF<R> U{reinterpret_cast<typename MatF<R>::S*>(const_cast<void*>(u))};
  if (adjoint_u)
    evaluate(O, adj(U) * I, n, st);
  else
    evaluate(O, U * I, n, st);
}

// host canonical (element-major, K complex128 per element) <-> blocked layout
template <class R>
void pack(std::vector<R>& dst, const double* src, int64_t n, int K) {
  const int64_t nb = (n + 63) / 64;
  dst.assign((size_t)nb * 64 * K * 2, (R)0);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < K; ++k) {
      const size_t o = (size_t)(((i >> 6) * K + k) * 64 + (i & 63)) * 2;
      dst[o] = (R)src[(i * K + k) * 2];
      dst[o + 1] = (R)src[(i * K + k) * 2 + 1];
    }
}
template <class R>
void unpack(double* dst, const std::vector<R>& src, int64_t n, int K) {
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < K; ++k) {
      const size_t o = (size_t)(((i >> 6) * K + k) * 64 + (i & 63)) * 2;
      dst[(i * K + k) * 2] = (double)src[o];
      dst[(i * K + k) * 2 + 1] = (double)src[o + 1];
    }
}

template <class R>
void to_device_t(void* dev, const double* host, int64_t n, int K, hipStream_t st) {
  std::vector<R> tmp;
  pack(tmp, host, n, K);
  LQ_HIP(hipMemcpyAsync(dev, tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice, st));
  LQ_HIP(hipStreamSynchronize(st));
}
template <class R>
void to_host_t(double* host, const void* dev, int64_t n, int K, hipStream_t st) {
  const int64_t nb = (n + 63) / 64;
  std::vector<R> tmp((size_t)nb * 64 * K * 2);
  LQ_HIP(hipMemcpyAsync(tmp.data(), dev, tmp.size() * sizeof(R), hipMemcpyDeviceToHost, st));
  LQ_HIP(hipStreamSynchronize(st));
  unpack(host, tmp, n, K);
}

}  // namespace

extern "C" {

size_t lq_site_array_bytes(int64_t n, int kind, int prec) {
  if (n < 0 || !prec_ok(prec) || (kind != LQ_SITE_SU3 && kind != LQ_SITE_SPINOR)) return 0;
  const int K = kind == LQ_SITE_SU3 ? 9 : 12;
  return (size_t)((n + 63) / 64) * 64 * K * (prec == LQ_F64 ? 16 : 8);
}

lq_status lq_site_array_to_device(void* dev, const double* host, int64_t n, int kind, int prec,
                                  void* stream) {
  if (!dev || !host || n < 0 || !prec_ok(prec) || (kind != LQ_SITE_SU3 && kind != LQ_SITE_SPINOR))
    return LQ_EINVAL;
  const int K = kind == LQ_SITE_SU3 ? 9 : 12;
  auto st = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    if (prec == LQ_F64)
      to_device_t<double>(dev, host, n, K, st);
    else
      to_device_t<float>(dev, host, n, K, st);
  });
}

lq_status lq_site_array_to_host(double* host, const void* dev, int64_t n, int kind, int prec,
                                void* stream) {
  if (!dev || !host || n < 0 || !prec_ok(prec) || (kind != LQ_SITE_SU3 && kind != LQ_SITE_SPINOR))
    return LQ_EINVAL;
  const int K = kind == LQ_SITE_SU3 ? 9 : 12;
  auto st = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    if (prec == LQ_F64)
      to_host_t<double>(host, dev, n, K, st);
    else
      to_host_t<float>(host, dev, n, K, st);
  });
}

lq_status lq_su3_mul(void* dev_u, const void* dev_v, const void* dev_w, const void* dev_x,
                     int64_t n, int form, int prec, void* stream) {
  if (!dev_u || !dev_v || !dev_w || n < 0 || !prec_ok(prec) || form < LQ_SU3_VW ||
      form > LQ_SU3_VWX || (form == LQ_SU3_VWX && !dev_x))
    return LQ_EINVAL;
  auto st = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    if (prec == LQ_F64)
      su3_mul_t<double>(dev_u, dev_v, dev_w, dev_x, n, form, st);
    else
      su3_mul_t<float>(dev_u, dev_v, dev_w, dev_x, n, form, st);
  });
}

lq_status lq_su3_spinor_mul(void* dev_out, const void* dev_u, const void* dev_in, int64_t n,
                            int adjoint_u, int prec, void* stream) {
  if (!dev_out || !dev_u || !dev_in || n < 0 || !prec_ok(prec)) return LQ_EINVAL;
  auto st = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    if (prec == LQ_F64)
      su3_spinor_t<double>(dev_out, dev_u, dev_in, n, adjoint_u, st);
    else
      su3_spinor_t<float>(dev_out, dev_u, dev_in, n, adjoint_u, st);
  });
}

}  // extern "C"
