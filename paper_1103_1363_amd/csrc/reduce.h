// Single-pass global reductions in FP64.
//
// Each workgroup reduces its values with wavefront shuffles (64 lanes) and
// an LDS step across its waves, writes one partial per value, and takes a
// ticket from a device counter.  The workgroup that takes the last ticket
// sums all partials in block order (so the result does not depend on the
// order in which workgroups finish), runs a caller-supplied finaliser on
// the totals (for example to form CG's alpha and beta on the device) and
// resets the counter for the next launch.  The agent-scope fences make the
// partials written through other XCDs' L2 caches visible to that workgroup.
#pragma once

#include "lq_internal.h"

namespace lq {

struct RedBuf {
  double* part;       // RED_MAX_BLOCKS * RED_NVAL partial sums
  unsigned* counter;  // ticket counter, zero between launches
  double* result;     // RED_NVAL totals of the last launch
};

inline RedBuf red_buf(lq_ctx* ctx) {
  ensure_red(ctx);
  char* b = reinterpret_cast<char*>(ctx->red);
  RedBuf r;
  r.part = reinterpret_cast<double*>(b);
  r.counter = reinterpret_cast<unsigned*>(b + sizeof(double) * RED_MAX_BLOCKS * RED_NVAL);
  r.result = reinterpret_cast<double*>(b + sizeof(double) * RED_MAX_BLOCKS * RED_NVAL + 256);
  return r;
}
constexpr size_t RED_BYTES = sizeof(double) * RED_MAX_BLOCKS * RED_NVAL + 256 + 256;

template <int N>
__device__ __forceinline__ void wave_sum(double v[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
}

// Sum v over the workgroup; the total is valid in thread 0.
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

// Every thread of every workgroup must call this (no early return before it).
// fin(const double* tot) runs once, in thread 0 of the last workgroup.
template <int N, class Fin>
__device__ __forceinline__ void reduce_finalize(double v[N], const RedBuf& rb, Fin fin) {
  __shared__ double sh[N][16];
  __shared__ int is_last;
  block_sum<N>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) rb.part[(int64_t)blockIdx.x * N + k] = v[k];
    __threadfence();
    const unsigned prev = atomicAdd(rb.counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double t[N];
#pragma unroll
  for (int k = 0; k < N; ++k) t[k] = 0.0;
  // fixed assignment of partials to threads and a fixed tree: deterministic
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < N; ++k) t[k] += __builtin_nontemporal_load(&rb.part[(int64_t)b * N + k]);
  block_sum<N>(t, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) rb.result[k] = t[k];
    fin(t);
    __threadfence();
    *rb.counter = 0u;
  }
}

struct NoFin {
  __device__ void operator()(const double*) const {}
};

}  // namespace lq
