// Multi-right-hand-side hopping term on the matrix cores.
//
// Layout of a multi-RHS field (up to 16 right-hand sides, FP16 or FP32):
// per site the nrhs spinors are interleaved, colour-major inside a spinor:
//   data[(site * nrhs + r) * 12 + colour * 4 + spin],  FP16 norms[site * nrhs + r].
// A wavefront handles one site at a time for all right-hand sides.
//
// One hop of the hopping term maps the neighbour spinor psi (4 spins x 3
// colours, per RHS) to (1 - S gamma_mu) U' psi, U' the link or its adjoint.
// Its upper two spins are h' = P U' psi with P the 2 x 4 spin projector
// (rows s_h, entries 1 at s_in = s_h and a coefficient c in {+-1, +-i} at
// one lower spin), and its lower two spins follow from h' by the fixed
// reconstruction of the direction.  With real and imaginary parts
// separated, h' for all RHS is one real product
//   h'[(a, s_h, re/im)][r] = sum_(b, s_in, re/im) A[(a, s_h, ro)][(b, s_in, ri)] psi[(b, s_in, ri)][r]
// of a 12 x 24 matrix A = real form of (P x U') and the 24 x nrhs block of
// neighbour spinors, which is the B operand exactly as stored (colour b of
// RHS r is 4 spins x (re, im) = 8 halves).  One v_mfma_f32_16x16x32_f16 per
// hop computes it; rows 12-15 and the K range 24-31 are zero padding.
//
// Operand layout of v_mfma_f32_16x16x32_f16 (lane l, i = l % 16,
// g = l / 16): A[i][8 g + j] and B[8 g + j][i] (j = 0..7, eight halves per
// lane), D[4 g + j][i] (j = 0..3).  With rows ordered (a, s_h, re/im) the
// lane (g, i) receives h' of colour a = g for RHS i, so the reconstruction,
// the per-site FP16 scale of each neighbour (applied to D in FP32) and the
// accumulation of the eight hops stay inside the lane.  A lane of the A
// operand needs one link element U'[a][b] (a gather of 4 bytes from an
// uncompressed FP16 copy of the links) and places it, in real form, at the
// two spin slots its row s_h selects: a permute, an xor and four selects.
//
// The clover epilogues use v_mfma_f32_16x16x16f16 on each 6 x 6 chirality
// block in the same lane layout (rows (a, spin-in-block, re/im), K groups
// colour): the lane holding colour a of RHS r supplies and receives the two
// spins of that block, again without data exchange between lanes.
#pragma once

#include <vector>

#include "dslash_core.h"
#include "reduce.h"
#include "solver_kernels.h"

namespace lq {

constexpr int MR_MAX = 16;  // right-hand sides per multi-RHS field

typedef _Float16 mr_half8 __attribute__((ext_vector_type(8)));
typedef _Float16 mr_half4 __attribute__((ext_vector_type(4)));
typedef _Float16 mr_half2 __attribute__((ext_vector_type(2)));
typedef float mr_float4 __attribute__((ext_vector_type(4)));
typedef unsigned mr_u4 __attribute__((ext_vector_type(4)));
typedef unsigned mr_u2 __attribute__((ext_vector_type(2)));

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

// FP16 copies of the operator for the multi-RHS kernels, site-major:
// links[((p * nsite + s) * 4 + mu) * 9 + 3 a + b] = U_mu(s)[a][b] of parity p
// (all nine entries), clover[s * 42 + 21 cb + k]: per chirality block the
// diagonal (d_k, 0) for k < 6, then the upper triangle in tri_idx order.
constexpr int MR_CLOV_SITE = 42;
constexpr int MR_CLOV_BLOCK = 21;

// half2 bit patterns: low half = real part, high half = imaginary part
constexpr unsigned MR_SGN_HI = 0x80000000u, MR_SGN_LO = 0x00008000u,
                   MR_SGN_BOTH = 0x80008000u;
constexpr unsigned MR_SEL_ID = 0x03020100u, MR_SEL_SWAP = 0x01000302u;  // v_perm_b32

__device__ __forceinline__ unsigned mr_perm(unsigned v, unsigned sel) {
  return __builtin_amdgcn_perm(v, v, sel);
}

// Load at a wave-uniform base plus a 32-bit per-lane byte offset (the
// scalar-base addressing form of global loads).
template <class T>
__device__ __forceinline__ T mr_ld(const void* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

// Lane constants of the A operands.  A row (a, s, ro) of the real form of
// a complex matrix z holds (Re z, -Im z) for ro = 0 and (Im z, Re z) for
// ro = 1 against the (re, im) parts of the K side; as half2 bits that is
// z ^ SGN_HI or swap(z), and for conj(z) it is z or swap(z) ^ SGN_LO.
struct MRLane {
  unsigned selX, selYi;  // selectors: real form of z, of i z
  unsigned mXf, mXb;     // xor masks: real form of z, of conj(z)
  unsigned mYf, mYb;     // xor masks: real form of i z, of i conj(z)
  unsigned msh;          // SGN_BOTH on rows with s_h = 1
  bool c0, c1;           // valid A row with s_h = 0 / s_h = 1
  unsigned ef, eb;       // byte offset of link entry U[a][b] / U[b][a]
  unsigned cslot[2];     // clover: byte offset of entry (k, l) for K spin 0 / 1
  unsigned cm[2];        // clover: xor mask of that entry (conjugated below the diagonal)
};

__device__ __forceinline__ MRLane mr_lane(int li, int grp) {
  MRLane q;
  const int a = li >> 2, sh = (li >> 1) & 1, ro = li & 1;
  const bool row = li < 12 && grp < 3;
  q.c0 = row && sh == 0;
  q.c1 = row && sh == 1;
  const int ac = a < 3 ? a : 0, bc = grp < 3 ? grp : 0;
  q.ef = (unsigned)(ac * 3 + bc) * 4u;
  q.eb = (unsigned)(bc * 3 + ac) * 4u;
  q.selX = ro ? MR_SEL_SWAP : MR_SEL_ID;
  q.selYi = ro ? MR_SEL_ID : MR_SEL_SWAP;
  q.mXf = ro ? 0u : MR_SGN_HI;
  q.mXb = ro ? MR_SGN_LO : 0u;
  q.mYf = ro ? MR_SGN_HI : MR_SGN_BOTH;
  q.mYb = ro ? 0u : MR_SGN_HI;
  q.msh = sh ? MR_SGN_BOTH : 0u;
  // clover rows (a_out, sib_out, ro) = (a, sh, ro); K (a_in = grp, sib_in, ri)
  const int k = sh * 3 + ac;
#pragma unroll
  for (int si = 0; si < 2; ++si) {
    const int l = si * 3 + bc;
    if (k == l) {
      q.cslot[si] = 4u * k;
      q.cm[si] = q.mXf;
    } else if (k < l) {
      q.cslot[si] = 4u * (6 + tri_idx(k, l));
      q.cm[si] = q.mXf;
    } else {
      q.cslot[si] = 4u * (6 + tri_idx(l, k));
      q.cm[si] = q.mXb;
    }
  }
  return q;
}

// One hop (direction MU, projector sign S, BACK: from x - mu with U^+) of
// the multi-RHS hopping term, given its gathered operands: v = the lane's
// link entry (half2 bits), B = the lane's 8 halves of neighbour spinor data,
// n = the neighbour's FP16 scale times the time boundary phase.  Builds the
// A operand, multiplies, and accumulates n * (upper, reconstructed lower
// spins) into acc[spin][re/im] of the lane's colour and RHS.
template <int MU, int S, bool BACK>
__device__ __forceinline__ void mr_hop1(unsigned v, mr_u4 B, float n, const MRLane& q,
                                        float acc[8]) {
  constexpr bool IMAG = (MU == 0 || MU == 2);     // c = +-i
  constexpr bool NEG = MU == 3 ? (S > 0) : (S < 0);  // sign of c on rows s_h = 0
  constexpr bool SHDEP = (MU == 1 || MU == 2);       // c changes sign with s_h
  const unsigned X = mr_perm(v, q.selX) ^ (BACK ? q.mXb : q.mXf);
  unsigned Y = IMAG ? (mr_perm(v, q.selYi) ^ (BACK ? q.mYb : q.mYf)) : X;
  if constexpr (NEG) Y ^= MR_SGN_BOTH;
  if constexpr (SHDEP) Y ^= q.msh;
  mr_u4 A;
  A[0] = q.c0 ? X : 0u;
  A[1] = q.c1 ? X : 0u;
  if constexpr (MU <= 1) {  // second slot 3 - s_h
    A[2] = q.c1 ? Y : 0u;
    A[3] = q.c0 ? Y : 0u;
  } else {  // second slot 2 + s_h
    A[2] = q.c0 ? Y : 0u;
    A[3] = q.c1 ? Y : 0u;
  }
  const mr_float4 z = {0.f, 0.f, 0.f, 0.f};
  const mr_float4 D = __builtin_amdgcn_mfma_f32_16x16x32_f16(
      __builtin_bit_cast(mr_half8, A), __builtin_bit_cast(mr_half8, B), z, 0, 0, 0);
  const float x0 = n * D[0], y0 = n * D[1], x1 = n * D[2], y1 = n * D[3];
  acc[0] += x0;
  acc[1] += y0;
  acc[2] += x1;
  acc[3] += y1;
  constexpr float sf = (float)S;
  if constexpr (MU == 0) {  // lower (-S i h1, -S i h0)
    acc[4] += sf * y1;
    acc[5] -= sf * x1;
    acc[6] += sf * y0;
    acc[7] -= sf * x0;
  } else if constexpr (MU == 1) {  // (-S h1, +S h0)
    acc[4] -= sf * x1;
    acc[5] -= sf * y1;
    acc[6] += sf * x0;
    acc[7] += sf * y0;
  } else if constexpr (MU == 2) {  // (-S i h0, +S i h1)
    acc[4] += sf * y0;
    acc[5] -= sf * x0;
    acc[6] -= sf * y1;
    acc[7] += sf * x1;
  } else {  // (-S h0, -S h1)
    acc[4] -= sf * x0;
    acc[5] -= sf * y0;
    acc[6] -= sf * x1;
    acc[7] -= sf * y1;
  }
}

// Chirality block cb of the clover table times the two spins (2 cb, 2 cb + 1)
// the lane holds as FP16 half2 bits in b, given the lane's two gathered
// table entries e (half2 bits): returns the lane's two output spins of its
// colour.
__device__ __forceinline__ mr_float4 mr_clover(const unsigned e[2], const MRLane& q, mr_u2 b) {
  const bool row = q.c0 || q.c1;
  mr_u2 A;
  A[0] = row ? (mr_perm(e[0], q.selX) ^ q.cm[0]) : 0u;
  A[1] = row ? (mr_perm(e[1], q.selX) ^ q.cm[1]) : 0u;
  const mr_float4 z = {0.f, 0.f, 0.f, 0.f};
  return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(mr_half4, A),
                                               __builtin_bit_cast(mr_half4, b), z, 0, 0, 0);
}

__device__ __forceinline__ unsigned mr_pack(float re, float im) {
  return __builtin_bit_cast(unsigned, mr_half2{(_Float16)re, (_Float16)im});
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
  void *p = nullptr, *q = nullptr, *t = nullptr;  // FP16 multi-RHS
  void *x = nullptr, *r = nullptr;                              // FP32 multi-RHS
  double* part = nullptr;   // per-block partials [blocks][MR_MAX]
  double* part2 = nullptr;  // first reduction stage [MR_ROWS2][MR_MAX]
  double* res = nullptr;   // totals
  MRState* st = nullptr;
  MRState* st_host = nullptr;
  std::vector<void*> b64, x64, bhat;  // per RHS FP64: full, full, even
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  double graph_k2 = 0;
};


enum {
  MR_EPI_NONE = 0,
  MR_EPI_CLOVINV = 1,
  MR_EPI_SCHUR2 = 2,
  MR_EPI_UPDATE = 3,
  MR_EPI_SCHUR2_F32 = 4  // as SCHUR2, the result stored in the FP32 field upd.r
};

// Operands of the CG update fused into the second Schur sweep
// (MR_EPI_UPDATE): x_r += alpha_r p_r and r_r -= alpha_r s_r with s the
// sweep's result, which is never stored.
struct MRUpd {
  MField<P32> x, r;
  MField<P16> p;
  const MRState* st;
};

// Eight halves (16 bytes) to floats.  The word is taken by value and split
// with shifts (element access through a reference to a vector in global
// memory read only its first element).
__device__ __forceinline__ void mr_h2f(const mr_u4 w, float f[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned u = w[k];
    f[2 * k] = (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xffffu));
    f[2 * k + 1] = (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
  }
}
constexpr int MR_BLK = 256;
#ifndef LQ_MR_SITES_PER_BLOCK
#define LQ_MR_SITES_PER_BLOCK 32
#endif
constexpr int MR_SITES_PER_BLOCK = LQ_MR_SITES_PER_BLOCK;  // 4 waves, each every 4th site

// out = H in (EPI_NONE), A^-1 H in (EPI_CLOVINV) or A x - k2 H in
// (EPI_SCHUR2, with per-workgroup partial |out|^2 per RHS in part[block][r]),
// for the sites of parity p of all right-hand sides.  EPI_UPDATE forms
// s = A x - k2 H in like EPI_SCHUR2 but, instead of storing it, applies the
// CG update of `upd` and writes the partial |r_new|^2 per RHS.
// EPI_SCHUR2_F32 forms A x - k2 H in like EPI_SCHUR2 and stores it in the
// FP32 field upd.r (no FP16 rounding; the block solver's Q).
// `active`: skip when 0.  links / clov: the FP16 site-major copies (clov:
// the table of parity p).
template <bool DAG, int EPI>
__global__ __launch_bounds__(MR_BLK) void mrhs_hop_kernel(
    Geo g, int p, const int* __restrict__ active, MField<P16> out, MField<P16> in,
    MField<P16> x, const unsigned* __restrict__ links, const unsigned* __restrict__ clov,
    const int* __restrict__ nbr, float k2, double* __restrict__ part, MRUpd upd) {
  constexpr bool AXPY =
      EPI == MR_EPI_SCHUR2 || EPI == MR_EPI_UPDATE || EPI == MR_EPI_SCHUR2_F32;  // A x - k2 H in
  __shared__ double red[4][MR_MAX];
  if (active && !*active) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, grp = lane >> 4;
  const int nrhs = in.nrhs;
  const MRLane q = mr_lane(li, grp);
  const bool bl = grp < 3 && li < nrhs;  // lane holds colour grp of RHS li
  // Lanes outside the batch (li >= nrhs, grp = 3) read a valid column and
  // colour (finite data): their K range has zero A entries and their D
  // columns are never stored.
  const int lic = li < nrhs ? li : nrhs - 1, grc = grp < 3 ? grp : 2;
  const unsigned bofs = (unsigned)(lic * 12 + grc * 4) * 4u;  // lane byte offset in a site's RHS block
  const unsigned* ind = reinterpret_cast<const unsigned*>(in.d);
  const int64_t nsite = g.nblk * 64;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  constexpr int SF = DAG ? -1 : 1;
  constexpr int NIT = MR_SITES_PER_BLOCK / 4;
  const int sblk = nrhs * 12;  // dwords per site of a multi-RHS field
  const int* nbase = nbr + (int64_t)p * nsite * 8;
  double nsum = 0.0;
  int64_t s = blk * MR_SITES_PER_BLOCK + wave;
  // neighbour rows are read one site ahead (scalar loads)
  int nt[8];
#pragma unroll
  for (int h = 0; h < 8; ++h) nt[h] = s < g.vh ? nbase[s * 8 + h] : 0;
  for (int it = 0; it < NIT; ++it, s += 4) {
    if (s >= g.vh) break;  // uniform across the wavefront
    int sy[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) sy[h] = nt[h] & 0x7fffffff;
    const bool tf = nt[6] < 0, tb = nt[7] < 0;  // hops across the antiperiodic time boundary
    if (it + 1 < NIT && s + 4 < g.vh) {
#pragma unroll
      for (int h = 0; h < 8; ++h) nt[h] = nbase[(s + 4) * 8 + h];
    }
    // gather every operand of the site first (one memory round trip).  The
    // neighbour spinor blocks are one 16-byte load per hop; the small
    // operands (8 x nrhs neighbour scales, the 72 link entries, the 42
    // clover words) are fetched with lane-dense loads, one word per lane,
    // and each lane then picks its entries with a cross-lane permute: a
    // wavefront load costs texture-address cycles for all 64 lanes however
    // few distinct words it touches.
    // (the small loads are issued first: loads complete in issue order, so
    // the permutes below wait for them and not for the spinor blocks)
    // scales: lane l holds RHS (l & 7) [+ 8] of neighbour l >> 3
    const int dh = lane >> 3, dr = lane & 7;
    int sd = sy[0];
#pragma unroll
    for (int h = 1; h < 8; ++h) sd = dh == h ? sy[h] : sd;
    const float* nrow = in.norm + (int64_t)sd * nrhs;
    const float na = nrow[dr < nrhs ? dr : nrhs - 1];
    const float nbb = nrow[dr + 8 < nrhs ? dr + 8 : nrhs - 1];
    // links: forward links of the site (36 contiguous words), then the
    // backward links of mu = 0..3 at the neighbours (9 words each): words
    // 0..63 in the first load, the last 8 in the second
    const int64_t lbase = (int64_t)(1 - p) * nsite * 36;
    int64_t lw0;
    {
      const int j = lane - 36, mu = j / 9;
      int sb = sy[1];
      sb = mu == 1 ? sy[3] : sb;
      sb = mu == 2 ? sy[5] : sb;
      sb = mu == 3 ? sy[7] : sb;
      lw0 = lane < 36 ? ((int64_t)p * nsite + s) * 36 + lane : lbase + (int64_t)sb * 36 + j;
    }
    const unsigned lda = links[lw0];
    const unsigned ldb = links[lbase + (int64_t)sy[7] * 36 + 28 + (lane < 8 ? lane : 7)];
    // clover words of the site (two blocks of 21)
    unsigned cw = 0u;
    if constexpr (EPI != MR_EPI_NONE) cw = clov[s * MR_CLOV_SITE + (lane < 42 ? lane : 41)];
    // the x block
    mr_u4 xv = {0u, 0u, 0u, 0u};
    float xn = 0.f;
    if constexpr (AXPY) {
      xv = mr_ld<mr_u4>(reinterpret_cast<const unsigned*>(x.d) + s * sblk, bofs);
      xn = mr_ld<float>(x.norm + s * nrhs, 4u * (unsigned)lic);
    }
    mr_u4 bv[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) bv[h] = mr_ld<mr_u4>(ind + (int64_t)sy[h] * sblk, bofs);
    // distribute: the lane's scale of each neighbour, its link entries, its
    // clover entries
    float nb[8];
    unsigned lv[8];
    unsigned ce[2][2] = {{0u, 0u}, {0u, 0u}};
    {
      const int ln = lic & 7;
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const float a = __shfl(na, h * 8 + ln, 64), b = __shfl(nbb, h * 8 + ln, 64);
        nb[h] = lic < 8 ? a : b;
      }
      const int ef = (int)(q.ef >> 2), eb = (int)(q.eb >> 2);
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        lv[2 * mu] = __shfl(lda, 9 * mu + ef, 64);
        if (mu < 3) {
          lv[2 * mu + 1] = __shfl(lda, 36 + 9 * mu + eb, 64);
        } else {
          const unsigned a = __shfl(lda, 63, 64), b = __shfl(ldb, eb > 0 ? eb - 1 : 0, 64);
          lv[7] = eb == 0 ? a : b;
        }
      }
      if constexpr (EPI != MR_EPI_NONE) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int k = 0; k < 2; ++k)
            ce[cb][k] = __shfl(cw, MR_CLOV_BLOCK * cb + (int)(q.cslot[k] >> 2), 64);
      }
    }
    // keep the gather ahead of the arithmetic (the scheduler would otherwise
    // sink loads towards their uses and serialise the memory latency)
    __builtin_amdgcn_sched_barrier(0);
    float colmax = 0.f;
#pragma unroll
    for (int h = 0; h < 8; ++h) colmax = fmaxf(colmax, nb[h]);
    if (tf) nb[6] = -nb[6];
    if (tb) nb[7] = -nb[7];
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    mr_hop1<0, SF, false>(lv[0], bv[0], nb[0], q, acc);
    mr_hop1<0, -SF, true>(lv[1], bv[1], nb[1], q, acc);
    mr_hop1<1, SF, false>(lv[2], bv[2], nb[2], q, acc);
    mr_hop1<1, -SF, true>(lv[3], bv[3], nb[3], q, acc);
    mr_hop1<2, SF, false>(lv[4], bv[4], nb[4], q, acc);
    mr_hop1<2, -SF, true>(lv[5], bv[5], nb[5], q, acc);
    mr_hop1<3, SF, false>(lv[6], bv[6], nb[6], q, acc);
    mr_hop1<3, -SF, true>(lv[7], bv[7], nb[7], q, acc);
    // epilogue: y[spin][re/im] of colour grp, RHS li
    float y[8];
    if constexpr (EPI == MR_EPI_NONE) {
#pragma unroll
      for (int k = 0; k < 8; ++k) y[k] = acc[k];
    } else {
      mr_u2 xb[2];
      if constexpr (AXPY) {
        xb[0] = mr_u2{xv[0], xv[1]};
        xb[1] = mr_u2{xv[2], xv[3]};
      } else {
        // FP16 operand: the hop sum scaled by 1 / (largest neighbour scale)
        const float cs = scale_rcp(colmax);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          xb[cb] = mr_u2{mr_pack(cs * acc[4 * cb], cs * acc[4 * cb + 1]),
                         mr_pack(cs * acc[4 * cb + 2], cs * acc[4 * cb + 3])};
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const mr_float4 d = mr_clover(ce[cb], q, xb[cb]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if constexpr (AXPY)
            y[4 * cb + j] = xn * d[j] - k2 * acc[4 * cb + j];
          else
            y[4 * cb + j] = colmax * d[j];
        }
      }
    }
    if constexpr (EPI == MR_EPI_UPDATE) {
      // x += alpha p, r -= alpha s for the lane's colour and RHS: 8 floats
      // of x and r, 8 halves of p, all contiguous
      if (bl) {
        const int64_t e0 = (s * nrhs + li) * 12 + grp * 4;  // complex index
        float4* xp = reinterpret_cast<float4*>(upd.x.d + e0);
        float4* rp = reinterpret_cast<float4*>(upd.r.d + e0);
        const mr_u4 pw = *reinterpret_cast<const mr_u4*>(upd.p.d + e0);
        const float al = (float)upd.st->alpha[li];
        const float ap = al * upd.p.norm[s * nrhs + li];
        float4 x0 = xp[0], x1 = xp[1], r0 = rp[0], r1 = rp[1];
        float pf[8];
        mr_h2f(pw, pf);
        x0.x += ap * pf[0];
        x0.y += ap * pf[1];
        x0.z += ap * pf[2];
        x0.w += ap * pf[3];
        x1.x += ap * pf[4];
        x1.y += ap * pf[5];
        x1.z += ap * pf[6];
        x1.w += ap * pf[7];
        r0.x -= al * y[0];
        r0.y -= al * y[1];
        r0.z -= al * y[2];
        r0.w -= al * y[3];
        r1.x -= al * y[4];
        r1.y -= al * y[5];
        r1.z -= al * y[6];
        r1.w -= al * y[7];
        xp[0] = x0;
        xp[1] = x1;
        rp[0] = r0;
        rp[1] = r1;
        nsum += (double)r0.x * r0.x + (double)r0.y * r0.y + (double)r0.z * r0.z +
                (double)r0.w * r0.w + (double)r1.x * r1.x + (double)r1.y * r1.y +
                (double)r1.z * r1.z + (double)r1.w * r1.w;
      }
      continue;
    }
    if constexpr (EPI == MR_EPI_SCHUR2_F32) {
      // the lane's colour of its RHS, 4 spins x (re, im), unrounded
      if (bl) {
        const int64_t e0 = (s * nrhs + li) * 12 + grp * 4;  // complex index
        float4* op = reinterpret_cast<float4*>(upd.r.d + e0);
        op[0] = make_float4(y[0], y[1], y[2], y[3]);
        op[1] = make_float4(y[4], y[5], y[6], y[7]);
      }
      continue;
    }
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) mx = fmaxf(mx, fabsf(y[k]));
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    if (bl) {
      const float inv = scale_rcp(mx);
      mr_u4 o;
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = mr_pack(inv * y[2 * k], inv * y[2 * k + 1]);
      *reinterpret_cast<mr_u4*>(reinterpret_cast<char*>(reinterpret_cast<unsigned*>(out.d) +
                                                        s * sblk) + bofs) = o;
      if (grp == 0) out.norm[s * nrhs + li] = mx;
      if constexpr (EPI == MR_EPI_SCHUR2) {
        double n2 = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) n2 += (double)y[k] * y[k];
        nsum += n2;
      }
    }
  }
  if (AXPY && part) {
    // per-RHS totals: the three colour lanes of a column, then the four waves
    nsum += __shfl_xor(nsum, 16, 64);
    nsum += __shfl_xor(nsum, 32, 64);
    if (grp == 0) red[wave][li] = nsum;
    __syncthreads();
    if (threadIdx.x < (unsigned)MR_MAX) {  // columns past nrhs hold zeros
      const int r = threadIdx.x;
      part[blockIdx.x * MR_MAX + r] = red[0][r] + red[1][r] + red[2][r] + red[3][r];
    }
  }
}

}  // namespace lq
