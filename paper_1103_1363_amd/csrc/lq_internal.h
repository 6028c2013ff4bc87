// Internal declarations of the lq library: context, device layouts, the
// complex arithmetic and precision traits shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lq.h"

#define LQ_HD __host__ __device__
#include "field_index.h"
#include "site_index.h"

namespace lq {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  lq_status code;
  Error(lq_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define LQ_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::lq::Error(LQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LQ_CHECK(cond, code, msg)                     \
  do {                                                \
    if (!(cond)) throw ::lq::Error((code), (msg));    \
  } while (0)

// Reciprocal of an FP16 field's per-site (or per-site, per-RHS) scale m, the
// largest component magnitude: 0 when m is below the smallest normal FP32
// number.  Such components are far below any rounding level of the solvers
// (the fronts of point-source Krylov vectors reach it on large lattices) and
// are stored as zero; 1 / m of a denormal m would overflow to infinity.
__device__ __forceinline__ float scale_inv(float m) {
  return m >= 1.17549435e-38f ? 1.f / m : 0.f;
}
__device__ __forceinline__ float scale_rcp(float m) {  // the same, hardware reciprocal
  return m >= 1.17549435e-38f ? __builtin_amdgcn_rcpf(m) : 0.f;
}

// ---------------------------------------------------------------- complex
template <class R>
struct C {
  R re, im;
};
template <class R>
__device__ __forceinline__ C<R> cmk(R a, R b) { return C<R>{a, b}; }
template <class R>
__device__ __forceinline__ C<R> operator+(C<R> a, C<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ C<R> operator-(C<R> a, C<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ C<R> operator-(C<R> a) { return {-a.re, -a.im}; }
template <class R>
__device__ __forceinline__ C<R> operator*(C<R> a, C<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__device__ __forceinline__ C<R> operator*(R s, C<R> a) { return {s * a.re, s * a.im}; }
template <class R>
__device__ __forceinline__ C<R> conj(C<R> a) { return {a.re, -a.im}; }
template <class R>
__device__ __forceinline__ C<R> times_i(C<R> a) { return {-a.im, a.re}; }
// conj(a) * b
template <class R>
__device__ __forceinline__ C<R> cmul_conj(C<R> a, C<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class R>
__device__ __forceinline__ R norm2(C<R> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------- precision traits
// Register budget of the hopping kernels: at least this many waves per SIMD
// (512 / waves VGPRs per lane).  The compiler otherwise hoists all eight
// neighbour loads and trades occupancy for instruction-level parallelism,
// which loses on these bandwidth-bound kernels.
#ifndef LQ_WAVES_F64
#define LQ_WAVES_F64 2
#endif
#ifndef LQ_WAVES_F32
#define LQ_WAVES_F32 4
#endif
#ifndef LQ_WAVES_F16
#define LQ_WAVES_F16 3
#endif
#define LQ_HOP_KERNEL(P) \
  __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P::waves)))
// Storage type S, arithmetic type R.  FP16 fields hold fp16(value / scale)
// with one FP32 scale per site stored after the component array.
struct P64 {
  using R = double;
  using S = double2;
  static constexpr bool has_norm = false;
  static constexpr int id = LQ_F64;
  static constexpr int waves = LQ_WAVES_F64;  // minimum waves per SIMD of hopping kernels
};
struct P32 {
  using R = float;
  using S = float2;
  static constexpr bool has_norm = false;
  static constexpr int id = LQ_F32;
  static constexpr int waves = LQ_WAVES_F32;
};
struct P16 {
  using R = float;
  using S = __half2;
  static constexpr bool has_norm = true;
  static constexpr int id = LQ_F16;
  static constexpr int waves = LQ_WAVES_F16;
};

template <class P>
__device__ __forceinline__ C<typename P::R> ld(const typename P::S* p, int64_t i);
template <>
__device__ __forceinline__ C<double> ld<P64>(const double2* p, int64_t i) {
  double2 v = p[i];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ld<P32>(const float2* p, int64_t i) {
  float2 v = p[i];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ld<P16>(const __half2* p, int64_t i) {
  float2 v = __half22float2(p[i]);
  return {v.x, v.y};
}
// Streaming loads for data read exactly once per sweep (links, clover
// tables): the non-temporal hint lets L2 keep the spinors, which are read
// by eight neighbours, instead of the streamed tables.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u1;
template <class P>
__device__ __forceinline__ C<typename P::R> ldnt(const typename P::S* p, int64_t i);
template <>
__device__ __forceinline__ C<double> ldnt<P64>(const double2* p, int64_t i) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p) + i);
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ldnt<P32>(const float2* p, int64_t i) {
  const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p) + i);
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ldnt<P16>(const __half2* p, int64_t i) {
  const nt_u1 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u1*>(p) + i);
  __half2 h;
  __builtin_memcpy(&h, &v, 4);
  const float2 f = __half22float2(h);
  return {f.x, f.y};
}

template <class P>
__device__ __forceinline__ void st(typename P::S* p, int64_t i, C<typename P::R> v);
template <>
__device__ __forceinline__ void st<P64>(double2* p, int64_t i, C<double> v) {
  p[i] = make_double2(v.re, v.im);
}
template <>
__device__ __forceinline__ void st<P32>(float2* p, int64_t i, C<float> v) {
  p[i] = make_float2(v.re, v.im);
}
template <>
__device__ __forceinline__ void st<P16>(__half2* p, int64_t i, C<float> v) {
  p[i] = __floats2half2_rn(v.re, v.im);
}

typedef unsigned h16x4 __attribute__((ext_vector_type(4)));  // one chunk: 4 FP16 pairs
typedef float f32x4 __attribute__((ext_vector_type(4)));     // one chunk: 2 FP32 complex

// FP16 pair (bits) <-> complex
__device__ __forceinline__ C<float> h2_to_c(unsigned u) {
  __half2 h;
  __builtin_memcpy(&h, &u, 4);
  const float2 f = __half22float2(h);
  return {f.x, f.y};
}
__device__ __forceinline__ unsigned c_to_h2(float re, float im) {
  const __half2 h = __floats2half2_rn(re, im);
  unsigned u;
  __builtin_memcpy(&u, &h, 4);
  return u;
}

// The 6 stored FP16 pairs (rows 0 and 1) of a chunked FP16 link: one 16-byte
// and one 8-byte streaming load.
typedef unsigned h16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load_link16_raw(const __half2* __restrict__ gauge, int64_t nblk,
                                                int p, int mu, int64_t s, unsigned w[6]) {
  const unsigned* g = reinterpret_cast<const unsigned*>(gauge);
  const h16x4 a = __builtin_nontemporal_load(
      reinterpret_cast<const h16x4*>(g + link16_idx(nblk, p, mu, s, 0)));
  const h16x2 b = __builtin_nontemporal_load(
      reinterpret_cast<const h16x2*>(g + link16_idx(nblk, p, mu, s, 4)));
  w[0] = a.x;
  w[1] = a.y;
  w[2] = a.z;
  w[3] = a.w;
  w[4] = b.x;
  w[5] = b.y;
}

// The 12 FP16 pairs of site s of a chunked FP16 field (raw bits), and back.
__device__ __forceinline__ void load_chunks16(const __half2* d, int64_t s, unsigned v[12]) {
  const h16x4* q = reinterpret_cast<const h16x4*>(d);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const h16x4 w = q[chunk16_idx(s, k)];
    v[4 * k] = w.x;
    v[4 * k + 1] = w.y;
    v[4 * k + 2] = w.z;
    v[4 * k + 3] = w.w;
  }
}
__device__ __forceinline__ void store_chunks16(__half2* d, int64_t s, const unsigned v[12]) {
  h16x4* q = reinterpret_cast<h16x4*>(d);
#pragma unroll
  for (int k = 0; k < 3; ++k) q[chunk16_idx(s, k)] = h16x4{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
}

// The 12 components of site s of a chunked FP32 field, and back.
__device__ __forceinline__ void load_chunks32(const float2* d, int64_t s, C<float> v[12]) {
  const f32x4* q = reinterpret_cast<const f32x4*>(d);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const f32x4 w = q[chunk32_idx(s, k)];
    v[2 * k] = {w.x, w.y};
    v[2 * k + 1] = {w.z, w.w};
  }
}
__device__ __forceinline__ void store_chunks32(float2* d, int64_t s, const C<float> v[12]) {
  f32x4* q = reinterpret_cast<f32x4*>(d);
#pragma unroll
  for (int k = 0; k < 6; ++k)
    q[chunk32_idx(s, k)] = f32x4{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
}

// A device spinor field of one parity (and one right-hand side).
template <class P>
struct Field {
  typename P::S* d;
  float* norm;  // FP16 only: per-site scale
};

// bytes of one parity field of vh sites for precision prec
inline size_t parity_field_bytes(int64_t nblk, int prec) {
  int64_t n = nblk * SB;
  switch (prec) {
    case LQ_F64: return (size_t)n * 12 * 16;
    case LQ_F32: return (size_t)n * 12 * 8;
    default: return (size_t)n * 12 * 4 + (size_t)n * 4;
  }
}

template <class P>
__host__ __device__ inline Field<P> field_at(void* base, int64_t nblk) {
  Field<P> f;
  f.d = reinterpret_cast<typename P::S*>(base);
  f.norm = P::has_norm ? reinterpret_cast<float*>(reinterpret_cast<char*>(base) +
                                                  (size_t)nblk * SB * 12 * 4)
                       : nullptr;
  return f;
}

// Load the 12 components of site s (spin-major, colour-minor).
template <class P>
__device__ __forceinline__ void load_spinor(const Field<P>& f, int64_t s,
                                            C<typename P::R> v[12]) {
  if constexpr (P::has_norm) {
    unsigned u[12];
    load_chunks16(f.d, s, u);
    const float n = f.norm[s];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = n * h2_to_c(u[c]);
  } else if constexpr (P::id == LQ_F32) {
    load_chunks32(f.d, s, v);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = ld<P>(f.d, spin_idx(s, c));
  }
}
template <class P>
__device__ __forceinline__ void store_spinor(const Field<P>& f, int64_t s,
                                             C<typename P::R> v[12]) {
  if constexpr (P::has_norm) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    f.norm[s] = m;
    const float inv = scale_inv(m);
    unsigned u[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) u[c] = c_to_h2(inv * v[c].re, inv * v[c].im);
    store_chunks16(f.d, s, u);
  } else if constexpr (P::id == LQ_F32) {
    store_chunks32(f.d, s, v);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) st<P>(f.d, spin_idx(s, c), v[c]);
  }
}

// Load the 12 raw components of site s (FP16: without the scale) and the
// site scale (1 for FP64/FP32).
template <class P>
__device__ __forceinline__ typename P::R load_raw(const Field<P>& f, int64_t s,
                                                   C<typename P::R> v[12]) {
  if constexpr (P::has_norm) {
    unsigned u[12];
    load_chunks16(f.d, s, u);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = h2_to_c(u[c]);
    return f.norm[s];
  } else if constexpr (P::id == LQ_F32) {
    load_chunks32(f.d, s, v);
    return 1.f;
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = ld<P>(f.d, spin_idx(s, c));
    return (typename P::R)1;
  }
}

}  // namespace lq

// Host-side context, work spaces and the functions of each source file.
#include "lq_host.h"
