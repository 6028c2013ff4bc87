// Multi-right-hand-side operator and batched CG (up to 16 right-hand sides
// sharing every operator application; the hopping term runs on the matrix
// cores, see mrhs_kernels.h).
//
// Batched CG: independent CG recurrences on Mhat^+ Mhat x_r = Mhat^+ bhat_r,
// one per right-hand side, with per-RHS alpha/beta on the device.  The
// operator fields (p, q, t, s) are FP16 multi-RHS fields, the vectors x and
// r FP32 multi-RHS fields; the solutions are held in FP64 per RHS and
// refreshed by reliable updates (FP64 residual from the single-RHS FP64
// operator), triggered when any RHS's normal residual fell by delta since
// its last update.  A converged RHS is frozen (alpha = beta = 0).
#include <chrono>
#include <cmath>
#include <cstring>

#include "mrhs_kernels.h"
#include "solver_kernels.h"

namespace lq {

namespace {

// ---------------------------------------------------------------- layout kernels
// host canonical half field of RHS r (rank t among the parity's sites) ->
// multi-RHS field slot r
template <class P>
__global__ void mr_pack_kernel(Geo g, int parity, MField<P> f, const double2* __restrict__ src,
                               int r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.vh) return;
  int x[4];
  canonical_coords(g, 2 * t, x);
  x[0] += (parity + x[0] + x[1] + x[2] + x[3]) & 1;
  const int64_t s = cb_index(g, x);
  double2 v[12];  // host order spin * 3 + colour
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = src[t * 12 + c];
  double m = 0.0;
  if constexpr (P::has_norm) {
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmax(m, fmax(fabs(v[c].x), fabs(v[c].y)));
    f.norm[s * f.nrhs + r] = (float)m;
  }
  const double inv = P::has_norm ? (m > 0.0 ? 1.0 / m : 0.0) : 1.0;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double2 w = v[sp * 3 + a];
      if constexpr (P::has_norm) {
        __half2 h;
        h.x = __half((_Float16)(w.x * inv));
        h.y = __half((_Float16)(w.y * inv));
        f.d[mr_idx(s, f.nrhs, r, a * 4 + sp)] = h;
      } else {
        st<P>(f.d, mr_idx(s, f.nrhs, r, a * 4 + sp),
              C<typename P::R>{(typename P::R)w.x, (typename P::R)w.y});
      }
    }
}

template <class P>
__global__ void mr_unpack_kernel(Geo g, int parity, MField<P> f, double2* __restrict__ dst, int r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.vh) return;
  int x[4];
  canonical_coords(g, 2 * t, x);
  x[0] += (parity + x[0] + x[1] + x[2] + x[3]) & 1;
  const int64_t s = cb_index(g, x);
  const double n = P::has_norm ? (double)f.norm[s * f.nrhs + r] : 1.0;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const C<typename P::R> w = ld<P>(f.d, mr_idx(s, f.nrhs, r, a * 4 + sp));
      dst[t * 12 + sp * 3 + a] = make_double2(n * (double)w.re, n * (double)w.im);
    }
}

// Neighbour table of the multi-RHS kernels: for site s of parity p the
// device numbers of its eight neighbours (x+0, x-0, x+1, ..., x-3), with
// bit 31 set where the hop crosses the antiperiodic time boundary.
__global__ void mr_nbr_kernel(Geo g, int* __restrict__ out) {
  const int64_t nsite = g.nblk * 64;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (p, s)
  if (t >= 2 * nsite) return;
  const int p = t >= nsite ? 1 : 0;
  const int64_t s = t - p * nsite;
  int* o = out + t * 8;
  if (s >= g.vh) {  // padding sites: harmless in-range entries
    for (int h = 0; h < 8; ++h) o[h] = 0;
    return;
  }
  int l[4], tc[4];
  site_local(g, p, s, l, tc);
  const int x3 = tc[3] * g.T[3] + l[3];
  for (int mu = 0; mu < 4; ++mu) {
    const int64_t f = neighbour(g, s, l, tc, mu, true), b = neighbour(g, s, l, tc, mu, false);
    const bool ff = mu == 3 && g.apt && x3 == g.L[3] - 1;
    const bool fb = mu == 3 && g.apt && x3 == 0;
    o[2 * mu] = (int)f | (ff ? (int)0x80000000 : 0);
    o[2 * mu + 1] = (int)b | (fb ? (int)0x80000000 : 0);
  }
}

// FP16 site-major copy of the links: all nine entries of U_mu(s), row 2
// rebuilt from the FP64 compressed field.
__global__ void mr_links_kernel(Geo gm, Geo gs, const double2* __restrict__ g64,
                                unsigned* __restrict__ out) {
  const int64_t nsite = gm.nblk * 64;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (p, m, mu)
  if (t >= 2 * nsite * 4) return;
  const int mu = (int)(t & 3);
  const int64_t ps = t >> 2;
  const int p = ps >= nsite ? 1 : 0;
  const int64_t m = ps - p * nsite;
  if (m >= gm.vh) {  // padding sites
#pragma unroll
    for (int e = 0; e < 9; ++e) out[t * 9 + e] = 0u;
    return;
  }
  int x[4];
  site_coords(gm, p, m, x);
  C<double> u[9];
  load_link<P64>(g64, gs.nblk, p, mu, cb_index(gs, x), u);
#pragma unroll
  for (int e = 0; e < 9; ++e)
    out[t * 9 + e] =
        __builtin_bit_cast(unsigned, mr_half2{(_Float16)u[e].re, (_Float16)u[e].im});
}

// FP16 site-major copy of a clover table (36 complex per site: per block
// three packed diagonal pairs then the upper triangle) with the diagonal
// unpacked to (d_k, 0).
__global__ void mr_clov_kernel(Geo gm, Geo gs, int p, const double2* __restrict__ c64,
                               unsigned* __restrict__ out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= gm.nblk * 64) return;
  if (m >= gm.vh) {  // padding sites
#pragma unroll
    for (int k = 0; k < MR_CLOV_SITE; ++k) out[m * MR_CLOV_SITE + k] = 0u;
    return;
  }
  int x[4];
  site_coords(gm, p, m, x);
  const int64_t s = cb_index(gs, x);
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    unsigned* o = out + m * MR_CLOV_SITE + cb * MR_CLOV_BLOCK;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double2 v = c64[clov_idx(s, 18 * cb + (k >> 1))];
      o[k] = __builtin_bit_cast(unsigned, mr_half2{(_Float16)((k & 1) ? v.y : v.x), (_Float16)0});
    }
#pragma unroll
    for (int t = 0; t < 15; ++t) {
      const double2 v = c64[clov_idx(s, 18 * cb + 3 + t)];
      o[6 + t] = __builtin_bit_cast(unsigned, mr_half2{(_Float16)v.x, (_Float16)v.y});
    }
  }
}

// single-RHS device field (precision PS) <-> slot r of a multi-RHS field:
// dst_slot = a * src + b * dst_slot (to_slot) or single = a * slot + b * single.
// A zero coefficient drops its operand unread, so a = b = 0 clears the
// destination whatever the other memory holds.
// The single field and the slot hold the even sites, each in its own
// numbering (g, gm).
template <class PS, class PM>
__global__ void mr_axpby_slot_kernel(Geo g, Geo gm, MField<PM> m, Field<PS> f, int r, double a,
                                     double b, int to_slot) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.vh) return;
  int x[4];
  site_coords(g, LQ_EVEN, s, x);
  const int64_t ms = cb_index(gm, x);
  const double cf = to_slot ? a : b, cm = to_slot ? b : a;  // coefficients of single, slot
  C<typename PS::R> fv[12];  // spin * 3 + colour
  double fn = 0.0;
  if (cf != 0.0) fn = (double)load_raw<PS>(f, s, fv);
  const double mn = (cm != 0.0 && PM::has_norm) ? (double)m.norm[ms * m.nrhs + r] : 1.0;
  double re[12], im[12];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = sp * 3 + c;
      re[k] = 0.0;
      im[k] = 0.0;
      if (cf != 0.0) {
        re[k] += cf * fn * (double)fv[k].re;
        im[k] += cf * fn * (double)fv[k].im;
      }
      if (cm != 0.0) {
        const C<typename PM::R> w = ld<PM>(m.d, mr_idx(ms, m.nrhs, r, c * 4 + sp));
        re[k] += cm * mn * (double)w.re;
        im[k] += cm * mn * (double)w.im;
      }
    }
  if (to_slot) {
    double mx = 0.0;
    if constexpr (PM::has_norm) {
#pragma unroll
      for (int k = 0; k < 12; ++k) mx = fmax(mx, fmax(fabs(re[k]), fabs(im[k])));
      m.norm[ms * m.nrhs + r] = (float)mx;
    }
    const double inv = PM::has_norm ? (mx > 0.0 ? 1.0 / mx : 0.0) : 1.0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int k = sp * 3 + c;
        st<PM>(m.d, mr_idx(ms, m.nrhs, r, c * 4 + sp),
               C<typename PM::R>{(typename PM::R)(inv * re[k]), (typename PM::R)(inv * im[k])});
      }
  } else {
    C<typename PS::R> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = C<typename PS::R>{(typename PS::R)re[k], (typename PS::R)im[k]};
    store_spinor<PS>(f, s, o);
  }
}

struct MRFinAlpha {
  MRState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;
    for (int r = 0; r < st->nrhs; ++r) {
      const double qq = tot[r];
      st->qq[r] = qq;
      if (!st->on[r]) {
        st->alpha[r] = 0.0;
      } else if (!(qq > 0.0) || !isfinite(qq)) {
        st->alpha[r] = 0.0;
        st->reason = R_NAN;
        st->active = 0;
      } else {
        st->alpha[r] = st->rr[r] / qq;
      }
    }
  }
};

struct MRFinBeta {
  MRState* st;
  __device__ void operator()(const double* tot) const {
    if (!st->active) return;
    st->iter += 1;
    int reason = R_RUN;
    for (int r = 0; r < st->nrhs; ++r) {
      if (!st->on[r]) {
        st->beta[r] = 0.0;
        continue;
      }
      const double rr = tot[r];
      if (!isfinite(rr)) {
        reason = R_NAN;
        continue;
      }
      st->beta[r] = rr / st->rr[r];
      st->rr[r] = rr;
      if (rr <= st->target2[r] || (st->delta2 > 0.0 && rr < st->delta2 * st->rr_max[r]))
        reason = reason == R_RUN ? R_RELIABLE : reason;
      if (rr > st->rr_max[r]) st->rr_max[r] = rr;
    }
    if (reason == R_RUN && st->iter >= st->maxiter) reason = R_MAXITER;
    if (reason != R_RUN) {
      st->reason = reason;
      st->active = 0;
    }
  }
};

// Reductions of per-block, per-RHS partial sums part[row][MR_MAX] in two
// deterministic stages: mr_rows_kernel sums fixed contiguous ranges of rows
// (one range per workgroup), mr_finalize_kernel sums those (one workgroup)
// and applies the solver step.  Threads of the 256-thread reduction blocks
// are (column = tid % 16, lane = tid / 16).
__device__ __forceinline__ double mr_sum16(double v, double (*red)[MR_MAX]) {
  // sum over the 16 lanes of each column: in-wave (4 lanes) then across waves
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  const int c = threadIdx.x & 15, w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) < 16) red[w][c] = v;
  __syncthreads();
  return red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

constexpr int MR_ROWS2 = 256;      // rows after the first reduction stage
constexpr int MR_UPD_BLOCKS = 1024;  // workgroups of the batched vector updates

__global__ __launch_bounds__(256) void mr_rows_kernel(const double* __restrict__ in, int nrows,
                                                      double* __restrict__ out) {
  __shared__ double red[4][MR_MAX];
  const int c = threadIdx.x & 15, l = threadIdx.x >> 4;
  const int chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const int lo = blockIdx.x * chunk, hi = min(lo + chunk, nrows);
  double t = 0.0;
  for (int i = lo + l; i < hi; i += 16) t += in[(int64_t)i * MR_MAX + c];
  t = mr_sum16(t, red);
  if (threadIdx.x < 16) out[blockIdx.x * MR_MAX + c] = t;
}

template <class Fin>
__global__ __launch_bounds__(256) void mr_finalize_kernel(const double* __restrict__ part,
                                                          int nparts, double* result, Fin fin) {
  __shared__ double red[4][MR_MAX];
  __shared__ double tot[MR_MAX];
  const int c = threadIdx.x & 15, l = threadIdx.x >> 4;
  double t = 0.0;
  for (int i = l; i < nparts; i += 16) t += part[i * MR_MAX + c];
  t = mr_sum16(t, red);
  if (threadIdx.x < 16) {
    tot[c] = t;
    result[c] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) fin(tot);
}

// The batched vector kernel: threadIdx.x = RHS (16 lanes), threadIdx.y =
// site (16 per step), grid-stride over sites.  Per (site, RHS) the 12
// complex of an FP32 field are six 16-byte words, of an FP16 field three.
// p_r = r_r + beta_r p_r, stored in FP16 with a new per-(site, RHS) scale.
__global__ __launch_bounds__(256) void mr_p_update(Geo g, const MRState* __restrict__ mst,
                                                   MField<P16> p, MField<P32> rv) {
  const int r = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int nrhs = p.nrhs;
  if (!mst->active || r >= nrhs) return;
  const float be = (float)mst->beta[r];
  for (int64_t s = (int64_t)blockIdx.x * 16 + ty; s < g.vh; s += (int64_t)gridDim.x * 16) {
    const int64_t i0 = mr_idx(s, nrhs, r, 0);
    const float bp = be * p.norm[s * nrhs + r];
    const float4* rp = reinterpret_cast<const float4*>(rv.d + i0);
    mr_u4* pp = reinterpret_cast<mr_u4*>(p.d + i0);
    float o[24];
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float pf[8];
      const mr_u4 pw = pp[k];
      mr_h2f(pw, pf);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float4 rr = rp[2 * k + h];
        o[8 * k + 4 * h] = rr.x + bp * pf[4 * h];
        o[8 * k + 4 * h + 1] = rr.y + bp * pf[4 * h + 1];
        o[8 * k + 4 * h + 2] = rr.z + bp * pf[4 * h + 2];
        o[8 * k + 4 * h + 3] = rr.w + bp * pf[4 * h + 3];
      }
    }
#pragma unroll
    for (int k = 0; k < 24; ++k) mx = fmaxf(mx, fabsf(o[k]));
    const float inv = scale_inv(mx);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      mr_u4 wv;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        wv[j] = __builtin_bit_cast(unsigned, mr_half2{(_Float16)(inv * o[8 * k + 2 * j]),
                                                      (_Float16)(inv * o[8 * k + 2 * j + 1])});
      pp[k] = wv;
    }
    p.norm[s * nrhs + r] = mx;
  }
}

}  // namespace

// ---------------------------------------------------------------- host helpers
size_t mr_field_bytes(const lq_ctx* ctx, int nrhs) { return mrhs_field_bytes(ctx->geo.nblk, LQ_F16, nrhs); }

namespace {

int mr_hop_grid(const Geo& g) { return grid_for(g.vh, MR_SITES_PER_BLOCK); }

void mr_hop(lq_ctx* ctx, int p, int dag, int epi, const int* active, void* out, const void* in,
            const void* x, int nrhs, double* part, MRUpd upd = MRUpd{}) {
  const Geo& g = ctx->mr_geo;
  LQ_CHECK(ctx->mr_links_ok && ctx->mr_nbr && (epi == MR_EPI_NONE || ctx->mr_clov_ok),
           LQ_ESTATE, "multi-RHS operator tables not built");
  MField<P16> fo = mfield_at<P16>(out, g.nblk, nrhs);
  MField<P16> fi = mfield_at<P16>(const_cast<void*>(in), g.nblk, nrhs);
  MField<P16> fx = mfield_at<P16>(const_cast<void*>(x ? x : in), g.nblk, nrhs);
  auto* lk = reinterpret_cast<const unsigned*>(ctx->mr_links);
  auto* nb = reinterpret_cast<const int*>(ctx->mr_nbr);
  const unsigned* cl = nullptr;
  if (epi != MR_EPI_NONE) cl = reinterpret_cast<const unsigned*>(ctx->mr_clov[p]);
  const float k2 = (float)(ctx->clov.kappa * ctx->clov.kappa);
  const dim3 grid(mr_hop_grid(g)), blk(MR_BLK);
  // algorithmic bytes: 8 links (12 reals), in and out per RHS, clover table, x per RHS
  double sb = 8 * link_site_bytes(LQ_F16) + 2.0 * nrhs * spinor_site_bytes(LQ_F16);
  if (epi != MR_EPI_NONE) sb += clover_site_bytes(LQ_F16);
  if (epi == MR_EPI_SCHUR2 || epi == MR_EPI_UPDATE || epi == MR_EPI_SCHUR2_F32)
    sb += nrhs * spinor_site_bytes(LQ_F16);
  if (epi == MR_EPI_SCHUR2_F32)  // FP32 output in place of the FP16 one
    sb += nrhs * (spinor_site_bytes(LQ_F32) - spinor_site_bytes(LQ_F16));
  if (epi == MR_EPI_UPDATE)  // no output; x, r read and written, p read
    sb += nrhs * (4 * spinor_site_bytes(LQ_F32) - spinor_site_bytes(LQ_F16)) +
          nrhs * spinor_site_bytes(LQ_F16);
  ctx->bytes += sb * (double)g.vh;
#define LQ_MR_LAUNCH(D, E)                                                                    \
  hipLaunchKernelGGL((mrhs_hop_kernel<D, E>), grid, blk, 0, ctx->cur, g, p, active, fo, fi, fx, \
                     lk, cl, nb, k2, part, upd)
  if (epi == MR_EPI_UPDATE) {
    LQ_CHECK(dag && upd.st, LQ_EINVAL, "the fused update follows the adjoint Schur sweep");
    LQ_MR_LAUNCH(true, MR_EPI_UPDATE);
  } else if (epi == MR_EPI_SCHUR2_F32) {
    LQ_CHECK(dag && upd.r.d, LQ_EINVAL, "the FP32 output follows the adjoint Schur sweep");
    LQ_MR_LAUNCH(true, MR_EPI_SCHUR2_F32);
  } else if (dag) {
    if (epi == MR_EPI_NONE) LQ_MR_LAUNCH(true, MR_EPI_NONE);
    else if (epi == MR_EPI_CLOVINV) LQ_MR_LAUNCH(true, MR_EPI_CLOVINV);
    else LQ_MR_LAUNCH(true, MR_EPI_SCHUR2);
  } else {
    if (epi == MR_EPI_NONE) LQ_MR_LAUNCH(false, MR_EPI_NONE);
    else if (epi == MR_EPI_CLOVINV) LQ_MR_LAUNCH(false, MR_EPI_CLOVINV);
    else LQ_MR_LAUNCH(false, MR_EPI_SCHUR2);
  }
#undef LQ_MR_LAUNCH
  LQ_HIP(hipGetLastError());
}

}  // namespace

// q32 = Mhat^+ Mhat p, every RHS (block solvers): p and the work fields t
// (odd) and q1 (even) FP16 multi-RHS fields, q32 an FP32 multi-RHS field
// written unrounded by the last sweep
void mrhs_normal(lq_ctx* ctx, void* q32, const void* p, void* t, void* q1, int nrhs) {
  const Geo& g = ctx->mr_geo;
  mr_hop(ctx, LQ_ODD, 0, MR_EPI_CLOVINV, nullptr, t, p, nullptr, nrhs, nullptr);
  mr_hop(ctx, LQ_EVEN, 0, MR_EPI_SCHUR2, nullptr, q1, t, p, nrhs, nullptr);
  mr_hop(ctx, LQ_ODD, 1, MR_EPI_CLOVINV, nullptr, t, q1, nullptr, nrhs, nullptr);
  MRUpd out{};
  out.r = mfield_at<P32>(q32, g.nblk, nrhs);
  mr_hop(ctx, LQ_EVEN, 1, MR_EPI_SCHUR2_F32, nullptr, q1, t, q1, nrhs, nullptr, out);
}

void mrhs_pack(lq_ctx* ctx, void* dev, const double2* src_dev, int parity, int prec, int nrhs,
               int r) {
  const Geo& g = ctx->mr_geo;  // multi-RHS site numbering
  ctx->bytes += (double)g.vh * (192.0 + spinor_site_bytes(prec));
  if (prec == LQ_F16)
    hipLaunchKernelGGL(mr_pack_kernel<P16>, dim3(grid_for(g.vh, 256)), dim3(256), 0, ctx->cur, g,
                       parity, mfield_at<P16>(dev, g.nblk, nrhs), src_dev, r);
  else
    hipLaunchKernelGGL(mr_pack_kernel<P32>, dim3(grid_for(g.vh, 256)), dim3(256), 0, ctx->cur, g,
                       parity, mfield_at<P32>(dev, g.nblk, nrhs), src_dev, r);
  LQ_HIP(hipGetLastError());
}

void mrhs_unpack(lq_ctx* ctx, double2* dst_dev, const void* dev, int parity, int prec, int nrhs,
                 int r) {
  const Geo& g = ctx->mr_geo;  // multi-RHS site numbering
  ctx->bytes += (double)g.vh * (192.0 + spinor_site_bytes(prec));
  void* d = const_cast<void*>(dev);
  if (prec == LQ_F16)
    hipLaunchKernelGGL(mr_unpack_kernel<P16>, dim3(grid_for(g.vh, 256)), dim3(256), 0, ctx->cur,
                       g, parity, mfield_at<P16>(d, g.nblk, nrhs), dst_dev, r);
  else
    hipLaunchKernelGGL(mr_unpack_kernel<P32>, dim3(grid_for(g.vh, 256)), dim3(256), 0, ctx->cur,
                       g, parity, mfield_at<P32>(d, g.nblk, nrhs), dst_dev, r);
  LQ_HIP(hipGetLastError());
}

void mrhs_tables(lq_ctx* ctx, bool clover) {
  const Geo& g = ctx->mr_geo;
  const int64_t nsite = g.nblk * 64;
  LQ_CHECK(g.vh < ((int64_t)1 << 31), LQ_EINVAL, "lattice too large for the multi-RHS kernels");
  if (!ctx->mr_nbr) {  // depends on the geometry only
    LQ_HIP(hipMalloc(&ctx->mr_nbr, (size_t)nsite * 2 * 8 * 4));
    hipLaunchKernelGGL(mr_nbr_kernel, dim3(grid_for(2 * nsite, 256)), dim3(256), 0, ctx->cur, g,
                       (int*)ctx->mr_nbr);
    LQ_HIP(hipGetLastError());
  }
  if (!ctx->mr_links_ok) {
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    if (!ctx->mr_links) LQ_HIP(hipMalloc(&ctx->mr_links, (size_t)nsite * 2 * 4 * 9 * 4));
    const int64_t n = nsite * 2 * 4;
    hipLaunchKernelGGL(mr_links_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->cur, g,
                       ctx->geo, (const double2*)ctx->gauge[LQ_F64], (unsigned*)ctx->mr_links);
    LQ_HIP(hipGetLastError());
    ctx->mr_links_ok = true;
  }
  if (clover && !ctx->mr_clov_ok) {
    LQ_CHECK(ctx->clov.valid, LQ_ESTATE, "no clover term (call lq_set_clover)");
    const void* src[2] = {ctx->clov.a64[LQ_EVEN], ctx->clov.ainv64[LQ_ODD]};
    for (int p = 0; p < 2; ++p) {
      if (!ctx->mr_clov[p]) LQ_HIP(hipMalloc(&ctx->mr_clov[p], (size_t)nsite * MR_CLOV_SITE * 4));
      hipLaunchKernelGGL(mr_clov_kernel, dim3(grid_for(nsite, 256)), dim3(256), 0, ctx->cur, g,
                         ctx->geo, p, (const double2*)src[p], (unsigned*)ctx->mr_clov[p]);
      LQ_HIP(hipGetLastError());
    }
    ctx->mr_clov_ok = true;
  }
}

void free_mrhs_tables(lq_ctx* ctx) {
  if (ctx->mr_nbr) (void)hipFree(ctx->mr_nbr);
  ctx->mr_nbr = nullptr;
  if (ctx->mr_links) (void)hipFree(ctx->mr_links);
  for (void* c : ctx->mr_clov)
    if (c) (void)hipFree(c);
  ctx->mr_links = nullptr;
  ctx->mr_clov[0] = ctx->mr_clov[1] = nullptr;
  ctx->mr_links_ok = ctx->mr_clov_ok = false;
}

void mrhs_dslash(lq_ctx* ctx, void* out, const void* in, int out_parity, int dagger, int nrhs) {
  mrhs_tables(ctx, false);
  mr_hop(ctx, out_parity, dagger, MR_EPI_NONE, nullptr, out, in, nullptr, nrhs, nullptr);
}

void mrhs_schur(lq_ctx* ctx, void* out, const void* in, void* tmp, int dagger, int nrhs) {
  mrhs_tables(ctx, true);
  mr_hop(ctx, LQ_ODD, dagger, MR_EPI_CLOVINV, nullptr, tmp, in, nullptr, nrhs, nullptr);
  mr_hop(ctx, LQ_EVEN, dagger, MR_EPI_SCHUR2, nullptr, out, tmp, in, nrhs, nullptr);
}

// ---------------------------------------------------------------- batched CG
namespace {

template <class PS, class PM>
void slot_axpby(lq_ctx* ctx, void* mfield, int nrhs, void* single, int r, double a, double b,
                int to_slot) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * (spinor_site_bytes(PS::id) * (to_slot ? 1 : 2) +
                                spinor_site_bytes(PM::id) * (to_slot ? 2 : 1));
  hipLaunchKernelGGL((mr_axpby_slot_kernel<PS, PM>), dim3(grid_for(g.vh, 256)), dim3(256), 0,
                     ctx->cur, g, ctx->mr_geo, mfield_at<PM>(mfield, g.nblk, nrhs),
                     field_at<PS>(single, g.nblk), r, a, b, to_slot);
  LQ_HIP(hipGetLastError());
}

// partial rows (one per workgroup) -> MRState via the two reduction stages
template <class Fin>
void mr_reduce(lq_ctx* ctx, MRWork* w, int nrows, Fin fin) {
  hipLaunchKernelGGL(mr_rows_kernel, dim3(MR_ROWS2), dim3(256), 0, ctx->cur, w->part, nrows,
                     w->part2);
  hipLaunchKernelGGL(mr_finalize_kernel<Fin>, dim3(1), dim3(256), 0, ctx->cur, w->part2,
                     MR_ROWS2, w->res, fin);
}

void mr_launch_iteration(lq_ctx* ctx, MRWork* w) {
  const Geo& g = ctx->mr_geo;  // multi-RHS site numbering
  const int n = w->nrhs;
  const int* act = &w->st->active;
  mr_hop(ctx, LQ_ODD, 0, MR_EPI_CLOVINV, act, w->t, w->p, nullptr, n, nullptr);
  mr_hop(ctx, LQ_EVEN, 0, MR_EPI_SCHUR2, act, w->q, w->t, w->p, n, w->part);
  mr_reduce(ctx, w, mr_hop_grid(g), MRFinAlpha{w->st});
  mr_hop(ctx, LQ_ODD, 1, MR_EPI_CLOVINV, act, w->t, w->q, nullptr, n, nullptr);
  // s = Mhat^+ q, used at once: x += alpha p, r -= alpha s, partial |r|^2
  const MRUpd upd{mfield_at<P32>(w->x, g.nblk, n), mfield_at<P32>(w->r, g.nblk, n),
                  mfield_at<P16>(w->p, g.nblk, n), w->st};
  mr_hop(ctx, LQ_EVEN, 1, MR_EPI_UPDATE, act, w->q, w->t, w->q, n, w->part, upd);
  mr_reduce(ctx, w, mr_hop_grid(g), MRFinBeta{w->st});
  hipLaunchKernelGGL(mr_p_update, dim3(MR_UPD_BLOCKS), dim3(256), 0, ctx->cur, g, w->st,
                     mfield_at<P16>(w->p, g.nblk, n), mfield_at<P32>(w->r, g.nblk, n));
  LQ_HIP(hipGetLastError());
}

}  // namespace

MRWork* mrhs_work(lq_ctx* ctx, int nrhs) {
  MRWork* w = ctx->mrwork;
  if (w && w->nrhs != nrhs) {
    free_mrhs_work(ctx);
    w = nullptr;
  }
  if (!w) {
    w = new MRWork();
    ctx->mrwork = w;
    w->nrhs = nrhs;
    w->nblk = ctx->geo.nblk;
    const size_t f16 = mrhs_field_bytes(w->nblk, LQ_F16, nrhs);
    const size_t f32 = mrhs_field_bytes(w->nblk, LQ_F32, nrhs);
    for (void** pp : {&w->p, &w->q, &w->t}) LQ_HIP(hipMalloc(pp, f16));
    for (void** pp : {&w->x, &w->r}) LQ_HIP(hipMalloc(pp, f32));
    const size_t nparts = (size_t)std::max(grid_for(ctx->geo.vh, MR_SITES_PER_BLOCK),
                                           MR_UPD_BLOCKS);
    LQ_HIP(hipMalloc(&w->part, nparts * MR_MAX * sizeof(double)));
    LQ_HIP(hipMalloc(&w->part2, (size_t)MR_ROWS2 * MR_MAX * sizeof(double)));
    LQ_HIP(hipMalloc(&w->res, MR_MAX * sizeof(double)));
    LQ_HIP(hipMalloc(&w->st, sizeof(MRState)));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->st_host), sizeof(MRState),
                         hipHostMallocDefault));
    const size_t f64 = parity_field_bytes(w->nblk, LQ_F64);
    for (int r = 0; r < nrhs; ++r) {
      void *b = nullptr, *x = nullptr, *bh = nullptr;
      LQ_HIP(hipMalloc(&b, 2 * f64));
      LQ_HIP(hipMalloc(&x, 2 * f64));
      LQ_HIP(hipMalloc(&bh, f64));
      w->b64.push_back(b);
      w->x64.push_back(x);
      w->bhat.push_back(bh);
    }
  }
  return w;
}

void free_mrhs_work(lq_ctx* ctx) {
  MRWork* w = ctx->mrwork;
  if (!w) return;
  for (void* p : {w->p, w->q, w->t, w->x, w->r})
    if (p) (void)hipFree(p);
  if (w->part) (void)hipFree(w->part);
  if (w->part2) (void)hipFree(w->part2);
  if (w->res) (void)hipFree(w->res);
  if (w->st) (void)hipFree(w->st);
  if (w->st_host) (void)hipHostFree(w->st_host);
  for (auto* v : {&w->b64, &w->x64, &w->bhat})
    for (void* p : *v) (void)hipFree(p);
  if (w->graph) (void)hipGraphExecDestroy(w->graph);
  delete w;
  ctx->mrwork = nullptr;
}

// Run the batched iteration until an update is due; returns the state.
void mrhs_iterate(lq_ctx* ctx, MRWork* w, int check_every, bool use_graph) {
  if (!use_graph) {
    for (int i = 0; i < check_every; ++i) mr_launch_iteration(ctx, w);
    return;
  }
  if (!w->graph || w->graph_iters != check_every || w->graph_k2 != ctx->clov.kappa) {
    if (w->graph) {
      (void)hipGraphExecDestroy(w->graph);
      w->graph = nullptr;
    }
    hipGraph_t gr = nullptr;
    const double bytes0 = ctx->bytes;
    LQ_HIP(hipStreamBeginCapture(ctx->cur, hipStreamCaptureModeThreadLocal));
    try {
      for (int i = 0; i < check_every; ++i) mr_launch_iteration(ctx, w);
    } catch (...) {
      (void)hipStreamEndCapture(ctx->cur, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    ctx->bytes = bytes0;  // capture launches nothing; replays are counted by iteration
    LQ_HIP(hipStreamEndCapture(ctx->cur, &gr));
    hipError_t e = hipGraphInstantiate(&w->graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    LQ_HIP(e);
    w->graph_iters = check_every;
    w->graph_k2 = ctx->clov.kappa;
  }
  LQ_HIP(hipGraphLaunch(w->graph, ctx->cur));
}

void mrhs_state_upload(lq_ctx* ctx, MRWork* w) {
  LQ_HIP(hipMemcpyAsync(w->st, w->st_host, sizeof(MRState), hipMemcpyHostToDevice, ctx->cur));
}
void mrhs_state_download(lq_ctx* ctx, MRWork* w) {
  LQ_HIP(hipMemcpyAsync(w->st_host, w->st, sizeof(MRState), hipMemcpyDeviceToHost, ctx->cur));
  LQ_HIP(hipStreamSynchronize(ctx->cur));
}

// Bytes of one batched iteration per site (all RHS), for the accounting.
double mrhs_iteration_site_bytes(int nrhs) {
  const double L = link_site_bytes(LQ_F16), S = spinor_site_bytes(LQ_F16),
               C = clover_site_bytes(LQ_F16), S32 = spinor_site_bytes(LQ_F32);
  const double hop = 8 * L + 2.0 * nrhs * S + C;
  return 2 * hop                                  // two A^-1 H
         + (hop + nrhs * S)                       // A p - k2 H t (p read beside t)
         + (hop + nrhs * (4 * S32 + S))           // A q - k2 H^+ t, no output, fused with
                                                  // x += alpha p, r -= alpha s
         + nrhs * (S32 + 2 * S);                  // p = r + beta p
}

void mrhs_slot_from_single(lq_ctx* ctx, MRWork* w, void* mfield, int prec, void* single,
                           int r, double a, double b, int single_prec) {
  LQ_CHECK(single_prec == LQ_F64 || single_prec == LQ_F32, LQ_EINVAL,
           "slot sources are FP64 or FP32 fields");
  if (single_prec == LQ_F64) {
    if (prec == LQ_F16)
      slot_axpby<P64, P16>(ctx, mfield, w->nrhs, single, r, a, b, 1);
    else
      slot_axpby<P64, P32>(ctx, mfield, w->nrhs, single, r, a, b, 1);
  } else {
    if (prec == LQ_F16)
      slot_axpby<P32, P16>(ctx, mfield, w->nrhs, single, r, a, b, 1);
    else
      slot_axpby<P32, P32>(ctx, mfield, w->nrhs, single, r, a, b, 1);
  }
}
void mrhs_single_from_slot(lq_ctx* ctx, MRWork* w, void* mfield, int prec, void* single64,
                           int r, double a, double b) {
  if (prec == LQ_F16)
    slot_axpby<P64, P16>(ctx, mfield, w->nrhs, single64, r, a, b, 0);
  else
    slot_axpby<P64, P32>(ctx, mfield, w->nrhs, single64, r, a, b, 0);
}

}  // namespace lq
