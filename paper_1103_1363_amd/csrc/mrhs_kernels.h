// Multi-right-hand-side hopping term on the matrix cores.
//
// Layout of a multi-RHS field (up to 16 right-hand sides, FP16 or FP32):
// per site the nrhs spinors are interleaved, colour-major inside a spinor:
//   data[(site * nrhs + r) * 12 + colour * 4 + spin],  FP16 norms[site * nrhs + r].
// A wavefront handles one site at a time for all right-hand sides.
//
// For one site and one hop, the contribution to the output of every RHS is
//   out[s_out, a, r] += sum_{s_h, b} R[s_out, s_h] U'[a, b] h[s_h, b, r],
// with h the spin-projected neighbour (two spins), U' the link (or its
// adjoint) and R the 4x2 spin reconstruction (entries 0, +-1, +-i).  Written
// with real and imaginary parts separated this is a real (24 x 12) x
// (12 x nrhs) product: rows (a, s_out, re/im), columns r, contraction over
// (b, s_h, re/im).  Two v_mfma_f32_16x16x16f16 (rows 0-15 and 16-23) per
// hop accumulate all eight hops in FP32; the link and the reconstruction
// are folded into the A operand, the projected spinors form the B operand.
//
// Operand layouts of v_mfma_f32_16x16x16f16 (64 lanes, lane l, i = l % 16,
// g = l / 16): A[i][4g + j] and B[4g + j][i] (j = 0..3, one half4 per lane),
// D[4g + j][i] (one float4 per lane).  Here i is the RHS column for B and D,
// and the contraction group g is the colour b of the neighbour (g = 3 is
// zero padding).
#pragma once

#include <vector>

#include "dslash_core.h"
#include "reduce.h"
#include "solver_kernels.h"

namespace lq {

constexpr int MR_MAX = 16;  // right-hand sides per multi-RHS field

typedef _Float16 mr_half4 __attribute__((ext_vector_type(4)));
typedef float mr_float4 __attribute__((ext_vector_type(4)));

template <class P>
struct MField {
  typename P::S* d;
  float* norm;  // FP16 only
  int nrhs;
};

inline size_t mrhs_field_bytes(int64_t nblk, int prec, int nrhs) {
  const size_t n = (size_t)nblk * 64 * nrhs;
  return prec == LQ_F16 ? n * 12 * 4 + n * 4 : n * 12 * (prec == LQ_F32 ? 8 : 16);
}

template <class P>
inline MField<P> mfield_at(void* base, int64_t nblk, int nrhs) {
  MField<P> f;
  f.d = reinterpret_cast<typename P::S*>(base);
  f.norm = P::has_norm ? reinterpret_cast<float*>(reinterpret_cast<char*>(base) +
                                                  (size_t)nblk * 64 * nrhs * 12 * 4)
                       : nullptr;
  f.nrhs = nrhs;
  return f;
}

__host__ __device__ inline int64_t mr_idx(int64_t s, int nrhs, int r, int c) {
  return ((s * nrhs) + r) * 12 + c;
}

// Spin reconstruction coefficient R[s_out][s_h] of the hop in direction MU
// with projector sign S (see dslash_core.h); 0, +-1 or +-i.
template <int MU, int S>
__device__ __forceinline__ C<float> recon_coeff(int s_out, int s_h) {
  if (s_out < 2) return C<float>{s_out == s_h ? 1.f : 0.f, 0.f};
  const float sf = (float)S;
  if constexpr (MU == 0) {  // lower: (-S i h1, -S i h0)
    return (s_out == 2) == (s_h == 1) ? C<float>{0.f, -sf} : C<float>{0.f, 0.f};
  } else if constexpr (MU == 1) {  // (-S h1, +S h0)
    if (s_out == 2) return s_h == 1 ? C<float>{-sf, 0.f} : C<float>{0.f, 0.f};
    return s_h == 0 ? C<float>{sf, 0.f} : C<float>{0.f, 0.f};
  } else if constexpr (MU == 2) {  // (-S i h0, +S i h1)
    if (s_out == 2) return s_h == 0 ? C<float>{0.f, -sf} : C<float>{0.f, 0.f};
    return s_h == 1 ? C<float>{0.f, sf} : C<float>{0.f, 0.f};
  } else {  // (-S h0, -S h1)
    return (s_out - 2) == s_h ? C<float>{-sf, 0.f} : C<float>{0.f, 0.f};
  }
}

// Spin projection of one colour: p[spin] -> (h0, h1).
template <int MU, int S>
__device__ __forceinline__ void project1(const C<float> p[4], C<float>& h0, C<float>& h1) {
  if constexpr (MU == 0) {
    h0 = S > 0 ? p[0] + times_i(p[3]) : p[0] - times_i(p[3]);
    h1 = S > 0 ? p[1] + times_i(p[2]) : p[1] - times_i(p[2]);
  } else if constexpr (MU == 1) {
    h0 = S > 0 ? p[0] + p[3] : p[0] - p[3];
    h1 = S > 0 ? p[1] - p[2] : p[1] + p[2];
  } else if constexpr (MU == 2) {
    h0 = S > 0 ? p[0] + times_i(p[2]) : p[0] - times_i(p[2]);
    h1 = S > 0 ? p[1] - times_i(p[3]) : p[1] + times_i(p[3]);
  } else {
    h0 = S > 0 ? p[0] - p[2] : p[0] + p[2];
    h1 = S > 0 ? p[1] - p[3] : p[1] + p[3];
  }
}

// Neighbour of the local site (l, tc, x3) in direction MU (forward or
// backward) as a checkerboard index; `sign` is the antiperiodic time phase.
template <int MU, bool BACK>
__device__ __forceinline__ int64_t mr_neighbour(const Geo& g, const int l[4], const int tc[4],
                                                int x3, float& sign) {
  sign = 1.f;
  if constexpr (MU == 3) {
    if (g.apt && x3 == (BACK ? 0 : g.L[3] - 1)) sign = -1.f;
  }
  int y[4] = {tc[0] * g.T[0] + l[0], tc[1] * g.T[1] + l[1], tc[2] * g.T[2] + l[2], x3};
  if constexpr (!BACK)
    y[MU] = (y[MU] + 1 == g.L[MU]) ? 0 : y[MU] + 1;
  else
    y[MU] = (y[MU] == 0) ? g.L[MU] - 1 : y[MU] - 1;
  return cb_index(g, y);
}

// One hop of the multi-RHS hopping term for site s with neighbour sy,
// accumulated into the two D tiles.  lane_i = lane % 16, g = lane / 16.
// `sc` scales the neighbour's FP16 data into the column scale of RHS lane_i
// (its stored norm times the time phase over the column scale), so that the
// B operand stays in [-2, 2] whatever the field's magnitude.
template <int MU, int S, bool BACK>
__device__ __forceinline__ void mrhs_hop_dir(const Geo& g, const MField<P16>& in,
                                             const __half2* __restrict__ gauge, int p, int64_t s,
                                             int64_t sy, float sc, int lane_i, int grp,
                                             mr_float4& acc0, mr_float4& acc1) {
  // B operand: projected neighbour spinor, colour b = grp, column = RHS lane_i
  mr_half4 B = {(_Float16)0, (_Float16)0, (_Float16)0, (_Float16)0};
  if (grp < 3 && lane_i < in.nrhs) {
    const int64_t base = mr_idx(sy, in.nrhs, lane_i, grp * 4);
    C<float> pv[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) pv[sp] = ld<P16>(in.d, base + sp);
    C<float> h0, h1;
    project1<MU, S>(pv, h0, h1);
    B = mr_half4{(_Float16)(sc * h0.re), (_Float16)(sc * h0.im), (_Float16)(sc * h1.re),
                 (_Float16)(sc * h1.im)};
  }
  // A operand: (R x U') in real form; rows m = (a * 4 + s_out) * 2 + re/im,
  // columns (b, s_h, re/im) with b = grp
  C<float> u[9];
  if constexpr (!BACK)
    load_link<P16>(gauge, g.nblk, p, MU, s, u);
  else
    load_link<P16>(gauge, g.nblk, 1 - p, MU, sy, u);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int m = lane_i + 16 * t;
    mr_half4 A = {(_Float16)0, (_Float16)0, (_Float16)0, (_Float16)0};
    if (m < 24 && grp < 3) {
      const int a = m >> 3, s_out = (m >> 1) & 3, ro = m & 1, b = grp;
      // U'[a][b]: U[a][b] forward, conj(U[b][a]) backward
      C<float> uab = {0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int ka = BACK ? k % 3 : k / 3, kb = BACK ? k / 3 : k % 3;
        if (ka == a && kb == b) uab = BACK ? conj(u[k]) : u[k];
      }
      float e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const C<float> z = recon_coeff<MU, S>(s_out, j >> 1) * uab;
        const int ri = j & 1;
        e[j] = ro == 0 ? (ri == 0 ? z.re : -z.im) : (ri == 0 ? z.im : z.re);
      }
      A = mr_half4{(_Float16)e[0], (_Float16)e[1], (_Float16)e[2], (_Float16)e[3]};
    }
    if (t == 0)
      acc0 = __builtin_amdgcn_mfma_f32_16x16x16f16(A, B, acc0, 0, 0, 0);
    else
      acc1 = __builtin_amdgcn_mfma_f32_16x16x16f16(A, B, acc1, 0, 0, 0);
  }
}

// Multiply one chirality block (6 complex, index spin_in_block * 3 + colour)
// by the clover table block cb of site s.
template <class P>
__device__ __forceinline__ void clover_block(const typename P::S* __restrict__ cl, int64_t s,
                                             int cb, const C<float> x[6], C<float> y[6]) {
  C<float> m[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const C<typename P::R> v = ldnt<P>(cl, clov_idx(s, 18 * cb + k));
    m[k] = C<float>{(float)v.re, (float)v.im};
  }
#pragma unroll
  for (int rr = 0; rr < 6; ++rr) {
    const float d = (rr & 1) ? m[rr >> 1].im : m[rr >> 1].re;
    C<float> acc = d * x[rr];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (c == rr) continue;
      if (rr < c)
        acc = acc + m[3 + tri_idx(rr, c)] * x[c];
      else
        acc = acc + cmul_conj(m[3 + tri_idx(c, rr)], x[c]);
    }
    y[rr] = acc;
  }
}

// State of the batched CG iteration (device, mirrored in pinned host memory).
struct MRState {
  double rr[MR_MAX];       // |r_r|^2 (normal residual, inner precision)
  double rr_max[MR_MAX];   // max since the last reliable update
  double target2[MR_MAX];  // inner stopping estimate for |r_r|^2
  double alpha[MR_MAX], beta[MR_MAX], qq[MR_MAX];
  double delta2;
  int on[MR_MAX];          // RHS still iterating
  int nrhs;
  int active;              // any RHS iterating and no update due
  int reason;              // R_RUN, R_RELIABLE (update due), R_NAN, R_MAXITER
  int iter, maxiter;
};


struct MRWork {
  int nrhs = 0;
  int64_t nblk = 0;
  void *p = nullptr, *q = nullptr, *t = nullptr, *s = nullptr;  // FP16 multi-RHS
  void *x = nullptr, *r = nullptr;                              // FP32 multi-RHS
  double* part = nullptr;  // per-block partials [blocks][MR_MAX]
  double* res = nullptr;   // totals
  MRState* st = nullptr;
  MRState* st_host = nullptr;
  std::vector<void*> b64, x64, bhat;  // per RHS FP64: full, full, even
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  double graph_k2 = 0;
};


enum { MR_EPI_NONE = 0, MR_EPI_CLOVINV = 1, MR_EPI_SCHUR2 = 2 };
constexpr int MR_BLK = 256;
constexpr int MR_SITES_PER_BLOCK = 32;  // 8 sites per wavefront

// out = H in (EPI_NONE), A^-1 H in (EPI_CLOVINV) or A x - k2 H in
// (EPI_SCHUR2, with per-workgroup partial |out|^2 per RHS in part[block][r]),
// for the sites of parity p of all right-hand sides.  `active`: skip when 0.
template <bool DAG, int EPI>
__global__ __launch_bounds__(MR_BLK) void mrhs_hop_kernel(
    Geo g, int p, const int* __restrict__ active, MField<P16> out, MField<P16> in,
    MField<P16> x, const __half2* __restrict__ gauge, const __half2* __restrict__ cl, float k2,
    double* __restrict__ part) {
  __shared__ C<float> stage[4][MR_MAX][12];
  __shared__ double red[4][MR_MAX];
  if (active && !*active) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lane_i = lane & 15, grp = lane >> 4;
  const int nrhs = in.nrhs;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  constexpr int SF = DAG ? -1 : 1;
  double nsum = 0.0;
  for (int it = 0; it < MR_SITES_PER_BLOCK / 4; ++it) {
    const int64_t s = blk * MR_SITES_PER_BLOCK + it * 4 + wave;
    if (s >= g.vh) break;  // uniform across the wavefront
    int l[4], tc[4];
    site_local(g, p, s, l, tc);
    const int x3 = tc[3] * g.T[3] + l[3];
    // neighbours, and the column scale of RHS lane_i: the largest of the
    // eight neighbour norms
    int64_t sy[8];
    float sg[8], nb[8];
    sy[0] = mr_neighbour<0, false>(g, l, tc, x3, sg[0]);
    sy[1] = mr_neighbour<0, true>(g, l, tc, x3, sg[1]);
    sy[2] = mr_neighbour<1, false>(g, l, tc, x3, sg[2]);
    sy[3] = mr_neighbour<1, true>(g, l, tc, x3, sg[3]);
    sy[4] = mr_neighbour<2, false>(g, l, tc, x3, sg[4]);
    sy[5] = mr_neighbour<2, true>(g, l, tc, x3, sg[5]);
    sy[6] = mr_neighbour<3, false>(g, l, tc, x3, sg[6]);
    sy[7] = mr_neighbour<3, true>(g, l, tc, x3, sg[7]);
    float colmax = 0.f;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      nb[h] = lane_i < nrhs ? in.norm[sy[h] * nrhs + lane_i] : 0.f;
      colmax = fmaxf(colmax, nb[h]);
    }
    const float cinv = colmax > 0.f ? 1.f / colmax : 0.f;
#pragma unroll
    for (int h = 0; h < 8; ++h) nb[h] *= sg[h] * cinv;
    mr_float4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    mrhs_hop_dir<0, SF, false>(g, in, gauge, p, s, sy[0], nb[0], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<0, -SF, true>(g, in, gauge, p, s, sy[1], nb[1], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<1, SF, false>(g, in, gauge, p, s, sy[2], nb[2], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<1, -SF, true>(g, in, gauge, p, s, sy[3], nb[3], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<2, SF, false>(g, in, gauge, p, s, sy[4], nb[4], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<2, -SF, true>(g, in, gauge, p, s, sy[5], nb[5], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<3, SF, false>(g, in, gauge, p, s, sy[6], nb[6], lane_i, grp, acc0, acc1);
    mrhs_hop_dir<3, -SF, true>(g, in, gauge, p, s, sy[7], nb[7], lane_i, grp, acc0, acc1);
    acc0 *= colmax;
    acc1 *= colmax;
    // D rows 4 grp .. 4 grp + 3 of column lane_i: two complex numbers
    // (colour a, spins sp, sp + 1) per tile
    if (lane_i < nrhs) {
      const int sp = 2 * (grp & 1);
      const int a0 = grp >> 1;
      stage[wave][lane_i][a0 * 4 + sp] = C<float>{acc0[0], acc0[1]};
      stage[wave][lane_i][a0 * 4 + sp + 1] = C<float>{acc0[2], acc0[3]};
      if (grp < 2) {
        stage[wave][lane_i][2 * 4 + sp] = C<float>{acc1[0], acc1[1]};
        stage[wave][lane_i][2 * 4 + sp + 1] = C<float>{acc1[2], acc1[3]};
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // epilogue: lane = 2 r + cb handles chirality block cb of RHS r
    const int r = lane >> 1, cb = lane & 1;
    const bool on = r < nrhs;
    C<float> hv[6], yv[6];
    if (on) {
#pragma unroll
      for (int k = 0; k < 6; ++k) hv[k] = stage[wave][r][(k % 3) * 4 + 2 * cb + k / 3];
      if constexpr (EPI == MR_EPI_NONE) {
#pragma unroll
        for (int k = 0; k < 6; ++k) yv[k] = hv[k];
      } else if constexpr (EPI == MR_EPI_CLOVINV) {
        clover_block<P16>(cl, s, cb, hv, yv);
      } else {
        C<float> xv[6];
        const float xn = x.norm[s * nrhs + r];
#pragma unroll
        for (int k = 0; k < 6; ++k)
          xv[k] = xn * ld<P16>(x.d, mr_idx(s, nrhs, r, (k % 3) * 4 + 2 * cb + k / 3));
        clover_block<P16>(cl, s, cb, xv, yv);
#pragma unroll
        for (int k = 0; k < 6; ++k) yv[k] = yv[k] - k2 * hv[k];
      }
    }
    float mx = 0.f;
    double n2 = 0.0;
    if (on) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        mx = fmaxf(mx, fmaxf(fabsf(yv[k].re), fabsf(yv[k].im)));
        n2 += (double)yv[k].re * yv[k].re + (double)yv[k].im * yv[k].im;
      }
    }
    mx = fmaxf(mx, __shfl_xor(mx, 1, 64));
    if (on) {
      const float inv = mx > 0.f ? 1.f / mx : 0.f;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        st<P16>(out.d, mr_idx(s, nrhs, r, (k % 3) * 4 + 2 * cb + k / 3), inv * yv[k]);
      if (cb == 0) out.norm[s * nrhs + r] = mx;
      nsum += n2;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (EPI == MR_EPI_SCHUR2 && part) {
    // per-RHS totals: pair the two chirality lanes, then the four waves
    nsum += __shfl_xor(nsum, 1, 64);
    if ((lane & 1) == 0 && (lane >> 1) < MR_MAX) red[wave][lane >> 1] = nsum;
    __syncthreads();
    if (threadIdx.x < (unsigned)nrhs) {
      const int r = threadIdx.x;
      part[blockIdx.x * MR_MAX + r] = red[0][r] + red[1][r] + red[2][r] + red[3][r];
    }
  }
}

}  // namespace lq
