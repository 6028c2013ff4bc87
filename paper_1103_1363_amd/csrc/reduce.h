// Global reductions in FP64, in two launches.
//
// The producing kernel reduces its per-site values inside each workgroup
// (wavefront shuffles over 64 lanes, then an LDS step across the waves) and
// writes one partial per value and workgroup.  A one-workgroup finalising
// kernel then sums the partials in a fixed order (the result does not
// depend on workgroup scheduling) and runs a caller-supplied finaliser on
// the totals, for example to form CG's alpha and beta on the device.
//
// A single-pass "last workgroup finishes" scheme was measured to halve the
// bandwidth of the producing kernels on MI355X: making each partial visible
// across the XCDs' separate L2 caches needs an agent-scope release per
// workgroup, which writes back the whole L2.  The kernel boundary provides
// that visibility once per launch instead.
#pragma once

#include "lq_internal.h"

namespace lq {

struct RedBuf {
  double* part;    // RED_MAX_BLOCKS * RED_NVAL partial sums
  double* result;  // RED_NVAL totals of the last reduction
};

inline RedBuf red_buf(lq_ctx* ctx) {
  ensure_red(ctx);
  char* b = reinterpret_cast<char*>(ctx->red);
  RedBuf r;
  r.part = reinterpret_cast<double*>(b);
  r.result = reinterpret_cast<double*>(b + sizeof(double) * RED_MAX_BLOCKS * RED_NVAL);
  return r;
}
constexpr size_t RED_BYTES = sizeof(double) * RED_MAX_BLOCKS * RED_NVAL + 256;

template <int N>
__device__ __forceinline__ void wave_sum(double v[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
}

// Sum v over the workgroup (at most 16 waves); the total is valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double v[N], double (*sh)[16]) {
  wave_sum<N>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[k][w];
      v[k] = s;
    }
}

// Every thread of every workgroup calls this (no early return before it).
template <int N>
__device__ __forceinline__ void block_partial(double v[N], double* part) {
  __shared__ double sh[N][16];
  block_sum<N>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[(int64_t)blockIdx.x * N + k] = v[k];
}

// As block_partial, at partial row idx instead of the workgroup index.
template <int N>
__device__ __forceinline__ void block_partial_at(double v[N], double* part, int64_t idx) {
  __shared__ double sh[N][16];
  block_sum<N>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[idx * N + k] = v[k];
}

// One workgroup: totals of nparts partials, then fin(totals) in thread 0.
template <int N, class Fin>
__global__ __launch_bounds__(256) void finalize_kernel(RedBuf rb, int nparts, Fin fin) {
  __shared__ double sh[N][16];
  double t[N];
#pragma unroll
  for (int k = 0; k < N; ++k) t[k] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < N; ++k) t[k] += rb.part[(int64_t)b * N + k];
  block_sum<N>(t, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) rb.result[k] = t[k];
    fin(t);
  }
}

struct NoFin {
  __device__ void operator()(const double*) const {}
};

}  // namespace lq
