// Fused site-local lattice expressions.
//
// Section 4 of the paper ports QDP++, a data-parallel library whose
// whole-lattice expressions (such as U_x = V_x W_x for every site x, eq.
// su3vecmul) are assembled from nested site types by templates, and which
// generates accelerator code for each expression an application uses.  Here
// the same idea targets gfx950: an expression over lattice fields builds a
// tree of types, and evaluate() instantiates one HIP kernel for that tree,
// so that an expression of any length reads each operand once and writes its
// result once (no temporaries, no extra passes over HBM).  The compiler's
// template instantiation plays the part of the paper's generator: every
// expression a program evaluates becomes a kernel of its own.
//
// Fields are device arrays of n elements in the library's blocked layout:
// component k of element i at ((i / 64) * K + k) * 64 + i % 64 (K complex
// components per element), so the 64 lanes of a wavefront read one component
// of 64 consecutive elements with one coalesced access.
//
// Site types (complex entries C<R>, R = double or float):
//   Mat<R>   3 x 3 colour matrix (row-major, K = 9)
//   Vec<R>   colour vector (K = 3)
//   Spin<R>  spinor, 4 spins x 3 colours (spin-major, K = 12)
// Operations: +, - on equal types; Mat * Mat, Mat * Vec, Mat * Spin (the
// matrix on every spin); complex scalar * any type; adj(Mat).
#pragma once

#include "lq_internal.h"

namespace lq {
namespace expr {

template <class R>
struct Mat {
  C<R> e[9];
};
template <class R>
struct Vec {
  C<R> e[3];
};
template <class R>
struct Spin {
  C<R> e[12];
};

template <class T>
struct ncomp;
template <class R>
struct ncomp<Mat<R>> {
  static constexpr int value = 9;
};
template <class R>
struct ncomp<Vec<R>> {
  static constexpr int value = 3;
};
template <class R>
struct ncomp<Spin<R>> {
  static constexpr int value = 12;
};

// ---------------------------------------------------------------- site arithmetic
template <class T>
__device__ __forceinline__ T add(const T& a, const T& b) {
  T r;
#pragma unroll
  for (int k = 0; k < ncomp<T>::value; ++k) r.e[k] = a.e[k] + b.e[k];
  return r;
}
template <class T>
__device__ __forceinline__ T sub(const T& a, const T& b) {
  T r;
#pragma unroll
  for (int k = 0; k < ncomp<T>::value; ++k) r.e[k] = a.e[k] - b.e[k];
  return r;
}
template <class T, class R>
__device__ __forceinline__ T scale(C<R> s, const T& a) {
  T r;
#pragma unroll
  for (int k = 0; k < ncomp<T>::value; ++k) r.e[k] = s * a.e[k];
  return r;
}
template <class R>
__device__ __forceinline__ Mat<R> mul(const Mat<R>& a, const Mat<R>& b) {
  Mat<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C<R> t = a.e[3 * i] * b.e[j];
      t = t + a.e[3 * i + 1] * b.e[3 + j];
      t = t + a.e[3 * i + 2] * b.e[6 + j];
      r.e[3 * i + j] = t;
    }
  return r;
}
template <class R>
__device__ __forceinline__ Vec<R> mul(const Mat<R>& a, const Vec<R>& v) {
  Vec<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    C<R> t = a.e[3 * i] * v.e[0];
    t = t + a.e[3 * i + 1] * v.e[1];
    t = t + a.e[3 * i + 2] * v.e[2];
    r.e[i] = t;
  }
  return r;
}
template <class R>
__device__ __forceinline__ Spin<R> mul(const Mat<R>& a, const Spin<R>& v) {
  Spin<R> r;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C<R> t = a.e[3 * i] * v.e[3 * s];
      t = t + a.e[3 * i + 1] * v.e[3 * s + 1];
      t = t + a.e[3 * i + 2] * v.e[3 * s + 2];
      r.e[3 * s + i] = t;
    }
  return r;
}
template <class R>
__device__ __forceinline__ Mat<R> adjoint(const Mat<R>& a) {
  Mat<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 * i + j] = conj(a.e[3 * j + i]);
  return r;
}

// ---------------------------------------------------------------- fields and nodes
// A lattice field of element type T in precision R (storage: double2 or float2).
template <class T, class R>
struct Field {
  using value_type = T;
  using S = typename std::conditional<std::is_same<R, double>::value, double2, float2>::type;
  S* d;
  __device__ __forceinline__ T eval(int64_t i) const {
    T v;
    const int64_t base = (i >> 6) * ncomp<T>::value * 64 + (i & 63);
#pragma unroll
    for (int k = 0; k < ncomp<T>::value; ++k) {
      const S x = d[base + (int64_t)k * 64];
      v.e[k] = C<R>{x.x, x.y};
    }
    return v;
  }
  __device__ __forceinline__ void store(int64_t i, const T& v) const {
    const int64_t base = (i >> 6) * ncomp<T>::value * 64 + (i & 63);
#pragma unroll
    for (int k = 0; k < ncomp<T>::value; ++k) {
      S x;
      x.x = v.e[k].re;
      x.y = v.e[k].im;
      d[base + (int64_t)k * 64] = x;
    }
  }
};

// Expression nodes.  Every node has value_type and eval(i).
template <class A, class B>
struct AddNode {
  using value_type = typename A::value_type;
  A a;
  B b;
  __device__ __forceinline__ value_type eval(int64_t i) const { return add(a.eval(i), b.eval(i)); }
};
template <class A, class B>
struct SubNode {
  using value_type = typename A::value_type;
  A a;
  B b;
  __device__ __forceinline__ value_type eval(int64_t i) const { return sub(a.eval(i), b.eval(i)); }
};
template <class A, class B, class V>
struct MulNode {
  using value_type = V;
  A a;
  B b;
  __device__ __forceinline__ value_type eval(int64_t i) const { return mul(a.eval(i), b.eval(i)); }
};
template <class A, class R>
struct ScaleNode {
  using value_type = typename A::value_type;
  C<R> s;
  A a;
  __device__ __forceinline__ value_type eval(int64_t i) const { return scale(s, a.eval(i)); }
};
template <class A>
struct AdjNode {
  using value_type = typename A::value_type;
  A a;
  __device__ __forceinline__ value_type eval(int64_t i) const { return adjoint(a.eval(i)); }
};

template <class X>
struct is_node : std::false_type {};
template <class T, class R>
struct is_node<Field<T, R>> : std::true_type {};
template <class A, class B>
struct is_node<AddNode<A, B>> : std::true_type {};
template <class A, class B>
struct is_node<SubNode<A, B>> : std::true_type {};
template <class A, class B, class V>
struct is_node<MulNode<A, B, V>> : std::true_type {};
template <class A, class R>
struct is_node<ScaleNode<A, R>> : std::true_type {};
template <class A>
struct is_node<AdjNode<A>> : std::true_type {};

template <class A, class B>
struct mul_type;
template <class R>
struct mul_type<Mat<R>, Mat<R>> {
  using type = Mat<R>;
};
template <class R>
struct mul_type<Mat<R>, Vec<R>> {
  using type = Vec<R>;
};
template <class R>
struct mul_type<Mat<R>, Spin<R>> {
  using type = Spin<R>;
};

template <class A, class B, class = std::enable_if_t<is_node<A>::value && is_node<B>::value>>
AddNode<A, B> operator+(const A& a, const B& b) {
  static_assert(std::is_same<typename A::value_type, typename B::value_type>::value,
                "sum of different site types");
  return {a, b};
}
template <class A, class B, class = std::enable_if_t<is_node<A>::value && is_node<B>::value>>
SubNode<A, B> operator-(const A& a, const B& b) {
  static_assert(std::is_same<typename A::value_type, typename B::value_type>::value,
                "difference of different site types");
  return {a, b};
}
template <class A, class B, class = std::enable_if_t<is_node<A>::value && is_node<B>::value>>
MulNode<A, B, typename mul_type<typename A::value_type, typename B::value_type>::type> operator*(
    const A& a, const B& b) {
  return {a, b};
}
template <class R, class A, class = std::enable_if_t<is_node<A>::value>>
ScaleNode<A, R> operator*(C<R> s, const A& a) {
  return {s, a};
}
template <class A, class = std::enable_if_t<is_node<A>::value>>
AdjNode<A> adj(const A& a) {
  return {a};
}

// ---------------------------------------------------------------- evaluation
template <class T, class R, class E>
__global__ __launch_bounds__(256) void eval_kernel(Field<T, R> dst, E e, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst.store(i, e.eval(i));
}

// dst = e over n elements, one fused kernel on `stream`.  dst may appear in e
// (each element is read before it is written, by the same thread).
template <class T, class R, class E>
void evaluate(const Field<T, R>& dst, const E& e, int64_t n, hipStream_t stream) {
  static_assert(std::is_same<T, typename E::value_type>::value, "assignment of another site type");
  if (n <= 0) return;
  hipLaunchKernelGGL((eval_kernel<T, R, E>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     stream, dst, e, n);
  LQ_HIP(hipGetLastError());
}

// Device bytes of a field of n elements of type T in precision R (whole
// 64-element blocks).
template <class T, class R>
inline size_t field_bytes(int64_t n) {
  return (size_t)((n + 63) / 64) * 64 * ncomp<T>::value * 2 * sizeof(R);
}

}  // namespace expr
}  // namespace lq
