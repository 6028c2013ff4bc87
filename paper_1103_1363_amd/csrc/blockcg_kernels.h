// Kernels of block CG on multi-RHS fields (K <= KM right-hand sides per
// site, interleaved: entry (s, r, c) at (s * K + r) * 12 + c; FP16 fields
// carry a scale per (s, r)).  The search block P is FP16 (the operator's
// input, used as rounded everywhere), Q = Mhat^+ Mhat P, X and R are FP32:
// rounding Q to FP16 as well breaks the block recurrence down.  A block vector is an N x K matrix with rows
// (site, component); the block method needs K x K Gram matrices A^H B of
// two such blocks, and the right multiplication of a block by a K x K
// matrix, fused into the passes that produce or consume the blocks:
//
//   bcg_gram:   G0 = P^H Q, G1 = P^H R (or Q^H Q, Q^H R)
//   bcg_update: X += P alpha, R -= Q alpha; then G0 = Q^H R, and |R_j|^2
//   bcg_dir:    W = R + P beta; then G0 = W^H W
//   bcg_orth:   P = W T (FP16 with per-(site, RHS) scales)
//
// A workgroup stages a tile of BT sites of each block it multiplies in LDS
// (rows (site, component) by KM columns) and forms its Gram contributions
// with register blocking: a thread owns one row i of the K x K result and
// four columns j0..j0+3, so each pair of LDS reads feeds four complex
// multiply-adds.  Products are FP32 within a tile, sums across tiles FP64;
// each workgroup writes its partial K x K matrices and a one-workgroup
// kernel per entry adds them in a fixed order.
#pragma once

#include "mrhs_kernels.h"

namespace lq {

#ifndef LQ_BCG_BT
#define LQ_BCG_BT 16
#endif
#ifndef LQ_BCG_GRID
#define LQ_BCG_GRID 2048
#endif
constexpr int BCG_BT = LQ_BCG_BT;      // sites per tile
constexpr int BCG_ROWS = BCG_BT * 12;
constexpr int BCG_THREADS = 256;
constexpr int BCG_GRID = LQ_BCG_GRID;  // workgroups (persistent over tiles)

// value of entry (s, r, c) as FP32 complex
template <class P>
__device__ __forceinline__ float2 bcg_ld(const MField<P>& f, int64_t s, int r, int c) {
  const int64_t i = ((s * f.nrhs) + r) * 12 + c;
  if constexpr (P::has_norm) {
    const float2 v = __half22float2(f.d[i]);
    const float n = f.norm[s * f.nrhs + r];
    return make_float2(n * v.x, n * v.y);
  } else {
    return f.d[i];
  }
}

// Stage rows of sites s0 .. s0 + ns - 1 of f into lds[row][KM] (zeros past K
// and past ns).
template <int KM, class P>
__device__ __forceinline__ void bcg_stage(const MField<P>& f, int64_t s0, int ns, float2* lds) {
  for (int e = threadIdx.x; e < BCG_BT * KM * 12; e += BCG_THREADS) {
    const int sl = e / (KM * 12), r = (e / 12) % KM, c = e % 12;
    float2 v = make_float2(0.f, 0.f);
    if (sl < ns && r < f.nrhs) v = bcg_ld<P>(f, s0 + sl, r, c);
    lds[(sl * 12 + c) * KM + r] = v;
  }
}

// Gram contributions of a staged tile: acc[j] += sum_rows conj(A[row][i]) B[row][j0 + j]
// for the thread's (i, j0), rows row0, row0 + stride, ...
template <int KM>
__device__ __forceinline__ void bcg_gram_tile(const float2* A, const float2* B, int i, int j0,
                                              int row0, int stride, double2 acc[4]) {
  float2 t[4] = {};
  for (int row = row0; row < BCG_ROWS; row += stride) {
    const float2 a = A[row * KM + i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 b = B[row * KM + j0 + j];
      t[j].x += a.x * b.x + a.y * b.y;
      t[j].y += a.x * b.y - a.y * b.x;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    acc[j].x += t[j].x;
    acc[j].y += t[j].y;
  }
}

// Thread roles of a Gram over NM matrices: (matrix, row i, column block) per
// thread within a group, GROUPS groups splitting the rows of each tile.
template <int KM, int NM>
struct BcgRole {
  static constexpr int PER = KM * (KM / 4);           // threads per matrix
  static constexpr int GROUPS = BCG_THREADS / (PER * NM);
  int m, i, j0, grp;
  bool on;
  __device__ BcgRole() {
    const int t = threadIdx.x;
    grp = t / (PER * NM);
    const int u = t % (PER * NM);
    m = u / PER;
    i = (u % PER) / (KM / 4);
    j0 = 4 * ((u % PER) % (KM / 4));
    on = grp < GROUPS;
  }
};

// Reduce the groups' accumulators and write the workgroup's partial
// matrices part[(blockIdx.x * NM + m) * KM * KM + i * KM + j] (double2).
template <int KM, int NM>
__device__ __forceinline__ void bcg_write_partial(const BcgRole<KM, NM>& ro, double2 acc[4],
                                                  double2* __restrict__ part, double2* red) {
  constexpr int PER = BcgRole<KM, NM>::PER, GROUPS = BcgRole<KM, NM>::GROUPS;
  __syncthreads();
  if (ro.on) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[(ro.grp * NM * KM + ro.m * KM + ro.i) * KM + ro.j0 + j] = acc[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NM * KM * KM; e += BCG_THREADS) {
    double2 s = make_double2(0.0, 0.0);
    for (int g = 0; g < GROUPS; ++g) {
      s.x += red[g * NM * KM * KM + e].x;
      s.y += red[g * NM * KM * KM + e].y;
    }
    part[(size_t)blockIdx.x * NM * KM * KM + e] = s;
  }
  (void)PER;
}

// G0 = A^H B, G1 = A^H C
template <int KM, class PA, class PB>
__global__ __launch_bounds__(BCG_THREADS) void bcg_gram_kernel(Geo g, MField<PA> p,
                                                               MField<PB> q, MField<P32> r,
                                                               double2* __restrict__ part) {
  __shared__ float2 sp[BCG_ROWS * KM], sq[BCG_ROWS * KM], sr[BCG_ROWS * KM];
  __shared__ double2 red[BcgRole<KM, 2>::GROUPS * 2 * KM * KM];
  const BcgRole<KM, 2> ro;
  double2 acc[4] = {};
  const int64_t ntile = (g.vh + BCG_BT - 1) / BCG_BT;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t s0 = tile * BCG_BT;
    const int ns = (int)min((int64_t)BCG_BT, g.vh - s0);
    __syncthreads();
    bcg_stage<KM>(p, s0, ns, sp);
    bcg_stage<KM>(q, s0, ns, sq);
    bcg_stage<KM>(r, s0, ns, sr);
    __syncthreads();
    if (ro.on)
      bcg_gram_tile<KM>(sp, ro.m == 0 ? sq : sr, ro.i, ro.j0, ro.grp, BcgRole<KM, 2>::GROUPS, acc);
  }
  bcg_write_partial<KM, 2>(ro, acc, part, red);
}

// X += P alpha, R -= Q alpha (alpha: K x K, entry (i, j) at alpha[i * KM + j]);
// then G0 = Q^H R (new R) and n2[j] = |R_j|^2 (as the diagonal of R^H R, G1)
template <int KM>
__global__ __launch_bounds__(BCG_THREADS) void bcg_update_kernel(
    Geo g, MField<P16> p, MField<P32> q, MField<P32> x, MField<P32> r,
    const float2* __restrict__ alpha, double2* __restrict__ part) {
  __shared__ float2 sq[BCG_ROWS * KM], sr[BCG_ROWS * KM];
  __shared__ float2 sa[KM * KM];
  __shared__ double2 red[BcgRole<KM, 2>::GROUPS * 2 * KM * KM];
  const int K = p.nrhs;
  for (int e = threadIdx.x; e < KM * KM; e += BCG_THREADS) sa[e] = alpha[e];
  const BcgRole<KM, 2> ro;
  double2 acc[4] = {};
  const int64_t ntile = (g.vh + BCG_BT - 1) / BCG_BT;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t s0 = tile * BCG_BT;
    const int ns = (int)min((int64_t)BCG_BT, g.vh - s0);
    __syncthreads();
    // one thread per row (site, component): all K columns of the row
    const int row = threadIdx.x;
    if (row < BCG_ROWS) {
      const int sl = row / 12, c = row % 12;
      float2 pv[KM], qv[KM];
#pragma unroll
      for (int i = 0; i < KM; ++i) {
        pv[i] = qv[i] = make_float2(0.f, 0.f);
        if (i < K && sl < ns) {
          pv[i] = bcg_ld<P16>(p, s0 + sl, i, c);
          qv[i] = bcg_ld<P32>(q, s0 + sl, i, c);
        }
      }
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        float2 rn = make_float2(0.f, 0.f);
        if (j < K && sl < ns) {
          const int64_t idx = (((s0 + sl) * K) + j) * 12 + c;
          float2 xv = x.d[idx], rv = r.d[idx];
#pragma unroll
          for (int i = 0; i < KM; ++i) {
            const float2 a = sa[i * KM + j];
            xv.x += pv[i].x * a.x - pv[i].y * a.y;
            xv.y += pv[i].x * a.y + pv[i].y * a.x;
            rv.x -= qv[i].x * a.x - qv[i].y * a.y;
            rv.y -= qv[i].x * a.y + qv[i].y * a.x;
          }
          x.d[idx] = xv;
          r.d[idx] = rv;
          rn = rv;
        }
        sr[row * KM + j] = rn;
        sq[row * KM + j] = qv[j];
      }
    }
    __syncthreads();
    if (ro.on)
      bcg_gram_tile<KM>(ro.m == 0 ? sq : sr, sr, ro.i, ro.j0, ro.grp, BcgRole<KM, 2>::GROUPS, acc);
  }
  bcg_write_partial<KM, 2>(ro, acc, part, red);
}

// W = R + P beta (W = R without reading P when with_p is 0: P holds nothing
// before the first search block); then G0 = W^H W
template <int KM>
__global__ __launch_bounds__(BCG_THREADS) void bcg_dir_kernel(Geo g, MField<P16> p,
                                                              MField<P32> r, MField<P32> w,
                                                              const float2* __restrict__ beta,
                                                              int with_p,
                                                              double2* __restrict__ part) {
  __shared__ float2 sw[BCG_ROWS * KM];
  __shared__ float2 sb[KM * KM];
  __shared__ double2 red[BcgRole<KM, 1>::GROUPS * KM * KM];
  const int K = p.nrhs;
  for (int e = threadIdx.x; e < KM * KM; e += BCG_THREADS) sb[e] = beta[e];
  const BcgRole<KM, 1> ro;
  double2 acc[4] = {};
  const int64_t ntile = (g.vh + BCG_BT - 1) / BCG_BT;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t s0 = tile * BCG_BT;
    const int ns = (int)min((int64_t)BCG_BT, g.vh - s0);
    __syncthreads();
    const int row = threadIdx.x;
    if (row < BCG_ROWS) {
      const int sl = row / 12, c = row % 12;
      float2 pv[KM];
#pragma unroll
      for (int i = 0; i < KM; ++i)
        pv[i] = (with_p && i < K && sl < ns) ? bcg_ld<P16>(p, s0 + sl, i, c)
                                             : make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        float2 wv = make_float2(0.f, 0.f);
        if (j < K && sl < ns) {
          const int64_t idx = (((s0 + sl) * K) + j) * 12 + c;
          wv = r.d[idx];
#pragma unroll
          for (int i = 0; i < KM; ++i) {
            const float2 b = sb[i * KM + j];
            wv.x += pv[i].x * b.x - pv[i].y * b.y;
            wv.y += pv[i].x * b.y + pv[i].y * b.x;
          }
          w.d[idx] = wv;
        }
        sw[row * KM + j] = wv;
      }
    }
    __syncthreads();
    if (ro.on) bcg_gram_tile<KM>(sw, sw, ro.i, ro.j0, ro.grp, BcgRole<KM, 1>::GROUPS, acc);
  }
  bcg_write_partial<KM, 1>(ro, acc, part, red);
}

// P = W T (T: K x K, entry (i, j) at t[i * KM + j]; columns past the rank
// are zero), stored in FP16 with a scale per (site, RHS)
template <int KM>
__global__ __launch_bounds__(BCG_THREADS) void bcg_orth_kernel(Geo g, MField<P32> w,
                                                               MField<P16> p,
                                                               const float2* __restrict__ t) {
  __shared__ float2 sw[BCG_ROWS * KM];
  __shared__ float2 st[KM * KM];
  const int K = p.nrhs;
  for (int e = threadIdx.x; e < KM * KM; e += BCG_THREADS) st[e] = t[e];
  const int64_t ntile = (g.vh + BCG_BT - 1) / BCG_BT;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t s0 = tile * BCG_BT;
    const int ns = (int)min((int64_t)BCG_BT, g.vh - s0);
    __syncthreads();
    bcg_stage<KM>(w, s0, ns, sw);
    __syncthreads();
    // one thread per (site, column j): the site's twelve components
    const int sl = threadIdx.x / KM, j = threadIdx.x % KM;
    if (sl < ns && j < K && threadIdx.x < BCG_BT * KM) {
      float2 v[12];
      float m = 0.f;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        float2 a = make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < KM; ++i) {
          const float2 wv = sw[(sl * 12 + c) * KM + i], tv = st[i * KM + j];
          a.x += wv.x * tv.x - wv.y * tv.y;
          a.y += wv.x * tv.y + wv.y * tv.x;
        }
        v[c] = a;
        m = fmaxf(m, fmaxf(fabsf(a.x), fabsf(a.y)));
      }
      const int64_t s = s0 + sl;
      p.norm[s * K + j] = m;
      const float inv = scale_inv(m);
#pragma unroll
      for (int c = 0; c < 12; ++c)
        p.d[(s * K + j) * 12 + c] = __floats2half2_rn(inv * v[c].x, inv * v[c].y);
    }
  }
}

// res[e] = sum over the nblocks partials of entry e (fixed order); one
// workgroup per entry
__global__ __launch_bounds__(256) void bcg_sum_kernel(const double2* __restrict__ part,
                                                      int nblocks, int nent,
                                                      double2* __restrict__ res) {
  __shared__ double sh[2][16];
  const int e = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    const double2 x = part[(size_t)b * nent + e];
    v[0] += x.x;
    v[1] += x.y;
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) res[e] = make_double2(v[0], v[1]);
}

}  // namespace lq
