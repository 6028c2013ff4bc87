// Uneven batch: independent even-odd Wilson-clover solves on lattices of
// different extents and hopping parameters, advanced together.
//
// The paper's solver (section 5: CG on the normal equations of the Schur
// operator, mixed precision by iterative refinement) is run for every member
// at once.  Each stage of an iteration is ONE kernel launch whose workgroups
// walk a tile list concatenated over the members still running: a workgroup
// finds its member from the tile index, loads that member's geometry,
// tables and fields from a device table, and skips the work when the
// member's iteration is not active.  The scalars of every member (CG's
// alpha, beta, residuals, stopping state) live on the device and are formed
// by one finalising launch with one workgroup per member, so small lattices
// (an 8^4 member has 2048 even sites, 8 workgroups) share the launches of
// the large ones instead of each paying its own launch and reduction
// latency.
//
// The FP64 reliable update (fold the inner correction into the FP64
// solution, recompute the Schur residual and the normal residual from the
// operator in FP64, restart the inner vectors from them) is also a fixed
// sequence of batched launches appended to every iteration; it acts only on
// the members whose iteration stopped in that iteration, so no host round
// trip is needed for it.  A captured graph replays check_every iterations;
// between replays the host reads the member states, and once a quarter of
// the tiles belong to finished members it rebuilds the tile list without
// them and captures again.  Members that broke down or stagnated are
// finished afterwards by the single-lattice solver (the FP64 fallback of
// solver.hip), from their current FP64 solution.
//
// A grid-wide-barrier persistent kernel was not used: every stage needs the
// previous stage's results from all XCDs, and a device-scope release per
// workgroup writes back the whole L2 of its XCD (reduce.h), which costs more
// than the kernel boundary of a graph-launched stage.
//
// Tile shape: sites per workgroup of the iteration kernels, chosen among
// 64, 128 and 256 by timing the iteration kernels on the members themselves,
// and cached per (GPU architecture, inner precision, nrhs, member extents),
// in memory and optionally in a JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "solver_kernels.h"

namespace lq {

constexpr int ENS_MAX = 64;     // members per batch
constexpr int UTB = 256;        // sites per tile of the update stage
constexpr int UGRID = 1024;     // workgroups of one update-stage launch at most
constexpr int STALL_ITERS = 200;
constexpr int TILE_CHOICES[3] = {64, 128, 256};

enum { E_RUN = 0, E_CONV = 1, E_MAXITER = 2, E_FALLBACK = 3 };

// Per-member solver state (device).
struct EState {
  CGState cg;
  int ru;           // 1: the update stage of this iteration acts on the member
  int done;         // E_*: 0 while the member still iterates
  int stalled;      // the iteration-level stagnation test stopped the iteration
  int updates;      // reliable updates completed (the initial residual excluded)
  int stall_iters;  // iterations without the inner residual quartering before
                    // giving up; 0 = no such test (FP64 inner iteration)
  int ref_iter;
  int nhist;
  int withhold;     // tests only: the fold drops the inner correction
  double ref_rt2;
  double hist[6];   // FP64 Schur residuals of the last reliable updates
};

// One member, as the kernels see it.
struct EMember {
  Geo g;
  int64_t t0, nt;  // iteration tiles: first index in the tile list, count
  int64_t r0, nr;  // update-stage tiles (UTB sites each)
  const void *gauge, *ainv, *aee;        // inner-precision tables
  const void *gauge64, *ainv64, *aee64;  // FP64 tables
  void *p, *q, *t, *xl, *r, *rt;         // inner iteration fields
  void *x, *bhat, *r64, *rn64, *to;      // FP64 fields (x: even half)
  EState* st;
  double k2;  // kappa^2
};

// ---------------------------------------------------------------- kernels
// Member of iteration tile b (uniform across the workgroup).
__device__ __forceinline__ int ens_member(const EMember* __restrict__ m, int nm, int64_t b) {
  int j = 0;
  while (j + 1 < nm && b >= m[j + 1].t0) ++j;
  return j;
}

#define ENS_HOP(P, TB) \
  __global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(P::waves)))

template <class PO, bool DAG, int TB>
ENS_HOP(PO, TB) void ens_k1(const EMember* __restrict__ m, int nm) {
  using S = typename PO::S;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const EMember& M = m[ens_member(m, nm, b)];
  if (!M.st->cg.active) return;
  const int64_t s = (b - M.t0) * TB + threadIdx.x;
  if (s >= M.g.vh) return;
  k1_site<PO, DAG>(M.g, s, field_at<PO>(M.t, M.g.nblk),
                   field_at<PO>(DAG ? M.q : M.p, M.g.nblk), (const S*)M.gauge,
                   (const S*)M.ainv);
}

template <class PO, int TB>
ENS_HOP(PO, TB) void ens_k2(const EMember* __restrict__ m, int nm, double* __restrict__ part) {
  using R = typename PO::R;
  using S = typename PO::S;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const EMember& M = m[ens_member(m, nm, b)];
  if (!M.st->cg.active) return;
  const int64_t s = (b - M.t0) * TB + threadIdx.x;
  double v[1] = {0.0};
  if (s < M.g.vh) {
    const int64_t nb = M.g.nblk;
    C<R> pv[12], y[12];
    schur_site<PO, false>(M.g, s, field_at<PO>(M.p, nb), field_at<PO>(M.t, nb),
                          (const S*)M.gauge, (const S*)M.aee, (R)M.k2, pv, y);
    store_spinor<PO>(field_at<PO>(M.q, nb), s, y);
    v[0] = site_norm2(y);
  }
  block_partial_at<1>(v, part, b);
}

template <class PO, class PV, int TB>
ENS_HOP(PO, TB) void ens_k4(const EMember* __restrict__ m, int nm, double* __restrict__ part) {
  using R = typename PO::R;
  using S = typename PO::S;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const EMember& M = m[ens_member(m, nm, b)];
  if (!M.st->cg.active) return;
  const int64_t s = (b - M.t0) * TB + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (s < M.g.vh) {
    const int64_t nb = M.g.nblk;
    C<R> qv[12], y[12];
    schur_site<PO, true>(M.g, s, field_at<PO>(M.q, nb), field_at<PO>(M.t, nb),
                         (const S*)M.gauge, (const S*)M.aee, (R)M.k2, qv, y);
    k4_update_site<PO, PV>(s, (R)M.st->cg.alpha, field_at<PO>(M.p, nb), field_at<PV>(M.xl, nb),
                           field_at<PV>(M.r, nb), field_at<PV>(M.rt, nb), y, qv, v);
  }
  block_partial_at<2>(v, part, b);
}

template <class PO, class PV, int TB>
__global__ __launch_bounds__(TB) void ens_k5(const EMember* __restrict__ m, int nm) {
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const EMember& M = m[ens_member(m, nm, b)];
  if (!M.st->cg.active) return;
  const int64_t s = (b - M.t0) * TB + threadIdx.x;
  if (s >= M.g.vh) return;
  k5_site<PO, PV>(s, (typename PO::R)M.st->cg.beta, field_at<PO>(M.p, M.g.nblk),
                  field_at<PV>(M.r, M.g.nblk));
}

// Totals of a member's partials of rows [r0, r0 + n), summed in a fixed
// order; valid in thread 0.
template <int N>
__device__ __forceinline__ void member_total(const double* __restrict__ part, int64_t r0,
                                             int64_t n, double t[N]) {
  __shared__ double sh[N][16];
#pragma unroll
  for (int k = 0; k < N; ++k) t[k] = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
    for (int k = 0; k < N; ++k) t[k] += part[(r0 + i) * N + k];
  block_sum<N>(t, sh);
}

// Members due an update stage, one bit per table slot: cleared by
// ens_fin_alpha, set by ens_fin_beta when a member's iteration stops, and
// cleared again by ens_fin_res for members that finished.  The update-stage
// kernels read this one word instead of every member's state.
using Mask = unsigned long long;

// One workgroup per member: alpha = |r|^2 / |Mhat p|^2.  Also ends the
// update stage of the previous iteration (clears ru and the mask).
__global__ __launch_bounds__(256) void ens_fin_alpha(const EMember* __restrict__ m,
                                                     const double* __restrict__ part,
                                                     Mask* __restrict__ due) {
  const EMember& M = m[blockIdx.x];
  double t[1];
  member_total<1>(part, M.t0, M.nt, t);
  if (threadIdx.x != 0) return;
  if (blockIdx.x == 0) *due = 0;
  EState* st = M.st;
  st->ru = 0;
  const int was = st->cg.active;
  FinAlpha{&st->cg}(t);
  if (was && !st->cg.active) st->done = E_FALLBACK;  // breakdown
}

// beta, convergence and reliable-update tests (FinBeta); a stop other than a
// breakdown schedules the update stage, as does the iteration-level
// stagnation test of the mixed-precision iteration.
__global__ __launch_bounds__(256) void ens_fin_beta(const EMember* __restrict__ m,
                                                    const double* __restrict__ part,
                                                    Mask* __restrict__ due) {
  const EMember& M = m[blockIdx.x];
  double t[2];
  member_total<2>(part, M.t0, M.nt, t);
  if (threadIdx.x != 0) return;
  EState* st = M.st;
  CGState& c = st->cg;
  if (!c.active) return;
  FinBeta{&c}(t);
  if (c.active) {
    if (c.rt2 <= 0.25 * st->ref_rt2) {
      st->ref_rt2 = c.rt2;
      st->ref_iter = c.iter;
    } else if (st->stall_iters > 0 && c.iter - st->ref_iter >= st->stall_iters) {
      c.active = 0;
      c.reason = R_RELIABLE;
      st->stalled = 1;
      st->ru = 1;
      atomicOr(due, Mask(1) << blockIdx.x);
    }
  } else if (c.reason == R_NAN) {
    st->done = E_FALLBACK;
  } else {
    st->ru = 1;
    atomicOr(due, Mask(1) << blockIdx.x);
  }
}

// Walks the update-stage tiles of the members whose bit is set in `due`, as
// one list of their tiles dealt round-robin to the workgroups; `body` gets
// the member, the site and the member's partial-sum row.  A launch with no
// member due returns after one load.
template <class Body>
__device__ __forceinline__ void update_tiles(const EMember* __restrict__ m, int nm,
                                             const Mask* __restrict__ due, Body body) {
  const Mask mk = *due;
  if (!mk) return;
  const int64_t G = gridDim.x;
  int64_t v0 = 0;  // list index of the current member's first tile
  for (int j = 0; j < nm; ++j) {
    if (!((mk >> j) & 1)) continue;
    const EMember& M = m[j];
    int64_t v = v0 + (((int64_t)blockIdx.x - v0) % G + G) % G;
    for (; v < v0 + M.nr; v += G) body(M, (v - v0) * UTB + threadIdx.x, M.r0 + (v - v0));
    v0 += M.nr;
  }
}

// x += xl (FP64), xl = 0
template <class PV>
__global__ __launch_bounds__(UTB) void ens_fold(const EMember* __restrict__ m, int nm,
                                                const Mask* __restrict__ due) {
  update_tiles(m, nm, due, [](const EMember& M, int64_t s, int64_t) {
    if (s >= M.g.vh) return;
    using RV = typename PV::R;
    const Field<P64> x = field_at<P64>(M.x, M.g.nblk);
    const Field<PV> xl = field_at<PV>(M.xl, M.g.nblk);
    C<double> a[12];
    C<RV> d[12];
    load_scaled<P64>(x, s, a);
    load_scaled<PV>(xl, s, d);
    const double keep = M.st->withhold ? 0.0 : 1.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      a[c] = a[c] + keep * C<double>{(double)d[c].re, (double)d[c].im};
      d[c] = C<RV>{(RV)0, (RV)0};
    }
    store_spinor<P64>(x, s, a);
    store_spinor<PV>(xl, s, d);
  });
}

// FP64 odd-site step: to = A_oo^-1 H_oe x (DAG: A_oo^-1 H^+_oe r64)
template <bool DAG>
__global__ __launch_bounds__(UTB) __attribute__((amdgpu_waves_per_eu(P64::waves)))
void ens_res_odd(const EMember* __restrict__ m, int nm, const Mask* __restrict__ due) {
  update_tiles(m, nm, due, [](const EMember& M, int64_t s, int64_t) {
    if (s >= M.g.vh) return;
    const int64_t nb = M.g.nblk;
    k1_site<P64, DAG>(M.g, s, field_at<P64>(M.to, nb), field_at<P64>(DAG ? M.r64 : M.x, nb),
                      (const double2*)M.gauge64, (const double2*)M.ainv64);
  });
}

// FP64 even-site step with partial sums:
//   !DAG: r64 = bhat - Mhat x,   partial |r64|^2
//    DAG: rn64 = Mhat^+ r64,     partial |rn64|^2
template <bool DAG>
__global__ __launch_bounds__(UTB) __attribute__((amdgpu_waves_per_eu(P64::waves)))
void ens_res_even(const EMember* __restrict__ m, int nm, const Mask* __restrict__ due,
                  double* __restrict__ part) {
  update_tiles(m, nm, due, [part](const EMember& M, int64_t s, int64_t b) {
    double v[1] = {0.0};
    if (s < M.g.vh) {
      const int64_t nb = M.g.nblk;
      C<double> in[12], y[12];
      schur_site<P64, DAG>(M.g, s, field_at<P64>(DAG ? M.r64 : M.x, nb), field_at<P64>(M.to, nb),
                           (const double2*)M.gauge64, (const double2*)M.aee64, M.k2, in, y);
      if constexpr (!DAG) {
        C<double> bh[12];
        load_scaled<P64>(field_at<P64>(M.bhat, nb), s, bh);
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = bh[c] - y[c];
        store_spinor<P64>(field_at<P64>(M.r64, nb), s, y);
      } else {
        store_spinor<P64>(field_at<P64>(M.rn64, nb), s, y);
      }
      v[0] = site_norm2(y);
    }
    block_partial_at<1>(v, part, b);
  });
}

// After the FP64 Schur residual: converged, out of iterations, stagnated
// (five updates without a factor-4 drop of |r|^2 after the oldest of six),
// or go on.
__global__ __launch_bounds__(256) void ens_fin_res(const EMember* __restrict__ m,
                                                   const double* __restrict__ part,
                                                   Mask* __restrict__ due) {
  const EMember& M = m[blockIdx.x];
  double t[1];
  member_total<1>(part, M.r0, M.nr, t);
  if (threadIdx.x != 0) return;
  EState* st = M.st;
  if (st->ru != 1) return;
  CGState& c = st->cg;
  const double rt2 = t[0];
  st->updates += 1;
  c.rt2 = rt2;
  c.rt2_max = rt2;
  int done = E_RUN;
  if (!isfinite(rt2)) {
    done = E_FALLBACK;
  } else if (rt2 <= c.target2) {
    done = E_CONV;
  } else if (st->stalled) {
    done = E_FALLBACK;
  } else if (c.reason == R_MAXITER || c.iter >= c.maxiter) {
    done = E_MAXITER;
  } else if (st->stall_iters > 0 && st->updates > 0) {
    if (st->nhist < 6) {
      st->hist[st->nhist++] = rt2;
    } else {
      for (int i = 0; i < 5; ++i) st->hist[i] = st->hist[i + 1];
      st->hist[5] = rt2;
    }
    if (st->nhist == 6) {
      double recent = st->hist[1];
      for (int i = 2; i < 6; ++i) recent = fmin(recent, st->hist[i]);
      if (recent > 0.25 * st->hist[0]) done = E_FALLBACK;
    }
  }
  st->done = done;
  if (done != E_RUN) atomicAnd(due, ~(Mask(1) << blockIdx.x));
}

// After the FP64 normal residual: restart the inner iteration.  The stopping
// iteration formed x, r and beta = |r_k+1|^2 / |r_k|^2 but not p_k+1; p goes
// on as r_new + (|r_new|^2 / |r_k|^2) p_k (beta = 0 at the first start).
__global__ __launch_bounds__(256) void ens_fin_rn(const EMember* __restrict__ m,
                                                  const double* __restrict__ part) {
  const EMember& M = m[blockIdx.x];
  double t[1];
  member_total<1>(part, M.r0, M.nr, t);
  if (threadIdx.x != 0) return;
  EState* st = M.st;
  if (st->ru != 1 || st->done != E_RUN) return;
  CGState& c = st->cg;
  const double rr_new = t[0];
  c.beta = (c.rr > 0.0 && c.beta > 0.0) ? c.beta * rr_new / c.rr : 0.0;
  c.rr = rr_new;
  c.active = 1;
  c.reason = R_RUN;
  if (c.rt2 <= 0.25 * st->ref_rt2) {
    st->ref_rt2 = c.rt2;
    st->ref_iter = c.iter;
  }
}

// r = rn64, rt = r64 (inner precision), p = r + beta p
template <class PO, class PV>
__global__ __launch_bounds__(UTB) void ens_load(const EMember* __restrict__ m, int nm,
                                                const Mask* __restrict__ due) {
  update_tiles(m, nm, due, [](const EMember& M, int64_t s, int64_t) {
    if (s >= M.g.vh) return;
    using R = typename PO::R;
    const int64_t nb = M.g.nblk;
    C<double> a[12];
    C<R> v[12];
    load_scaled<P64>(field_at<P64>(M.rn64, nb), s, a);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = C<R>{(R)a[c].re, (R)a[c].im};
    store_spinor<PV>(field_at<PV>(M.r, nb), s, v);
    k5_site<PO, PV>(s, (R)M.st->cg.beta, field_at<PO>(M.p, nb), field_at<PV>(M.r, nb));
    load_scaled<P64>(field_at<P64>(M.r64, nb), s, a);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = C<R>{(R)a[c].re, (R)a[c].im};
    store_spinor<PV>(field_at<PV>(M.rt, nb), s, v);
  });
}

// ---------------------------------------------------------------- host
struct TuneEntry {
  int tile = 0;
  bool from_cache = false;
  double ms[3] = {0, 0, 0};
};

struct Ensemble {
  std::vector<lq_ctx*> mem;
  hipStream_t stream = nullptr;
  EMember* table = nullptr;       // device
  EMember* table_host = nullptr;  // pinned
  EState* st = nullptr;           // device, one per member
  EState* st_host = nullptr;      // pinned
  double* part = nullptr;         // partial sums, one row per tile
  int64_t part_rows = 0;
  Mask* due = nullptr;            // device: members due an update stage
  Mask* due_host = nullptr;       // pinned
  hipGraphExec_t graph = nullptr;
  std::string graph_key;
  std::map<std::string, TuneEntry> tuned;
};

namespace {

const char* prec_name(int p) { return p == LQ_F64 ? "f64" : p == LQ_F32 ? "f32" : "f16"; }

std::string arch_name() {
  int dev = 0;
  LQ_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  LQ_HIP(hipGetDeviceProperties(&prop, dev));
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_key(const Ensemble* E, int inner) {
  std::ostringstream k;
  k << arch_name() << ":" << prec_name(inner) << ":nrhs1:";
  for (size_t j = 0; j < E->mem.size(); ++j) {
    const int* d = E->mem[j]->dims;
    k << (j ? "+" : "") << d[0] << "x" << d[1] << "x" << d[2] << "x" << d[3];
  }
  return k.str();
}

// The tile cache file: one JSON object whose members are
//   "<key>": {"tile_sites": N, "ms": [t64, t128, t256]}
// Entries of other keys are kept as they are when the file is rewritten.
std::map<std::string, std::string> read_cache(const std::string& path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = s.find('{');
  if (i == std::string::npos) return out;
  ++i;
  for (;;) {
    const size_t q0 = s.find('"', i);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
    const size_t o = s.find('{', q1);
    if (o == std::string::npos) break;
    int depth = 0;
    size_t e = o;
    for (; e < s.size(); ++e) {
      if (s[e] == '{') ++depth;
      if (s[e] == '}' && --depth == 0) break;
    }
    if (e >= s.size()) break;
    out[key] = s.substr(o, e - o + 1);
    i = e + 1;
  }
  return out;
}

bool parse_entry(const std::string& body, TuneEntry& t) {
  const size_t k = body.find("\"tile_sites\"");
  if (k == std::string::npos) return false;
  const size_t c = body.find(':', k);
  if (c == std::string::npos) return false;
  const int v = std::atoi(body.c_str() + c + 1);
  for (int x : TILE_CHOICES)
    if (v == x) {
      t.tile = v;
      const size_t a = body.find('[', c);
      if (a != std::string::npos) {
        std::istringstream in(body.substr(a + 1));
        for (int i = 0; i < 3; ++i) {
          char sep;
          if (!(in >> t.ms[i])) break;
          in >> sep;
        }
      }
      return true;
    }
  return false;
}

void write_cache(const std::string& path, const std::string& key, const TuneEntry& t) {
  std::map<std::string, std::string> all = read_cache(path);
  std::ostringstream e;
  e << "{\"tile_sites\": " << t.tile << ", \"ms\": [" << t.ms[0] << ", " << t.ms[1] << ", "
    << t.ms[2] << "]}";
  all[key] = e.str();
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    LQ_CHECK(f.good(), LQ_EINVAL, "cannot write the tile cache file " + path);
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : all)
      f << "  \"" << kv.first << "\": " << kv.second << (++n < all.size() ? ",\n" : "\n");
    f << "}\n";
    LQ_CHECK(f.good(), LQ_EINVAL, "cannot write the tile cache file " + path);
  }
  LQ_CHECK(std::rename(tmp.c_str(), path.c_str()) == 0, LQ_EINVAL,
           "cannot replace the tile cache file " + path);
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Fill the device table with the listed members; returns the iteration-tile
// and update-tile counts.
void build_table(Ensemble* E, int inner, int tb, const std::vector<int>& live, int64_t& ntiles,
                 int64_t& nutiles) {
  int64_t t0 = 0, r0 = 0;
  for (size_t i = 0; i < live.size(); ++i) {
    const int j = live[i];
    lq_ctx* c = E->mem[j];
    const SolveFields f = solve_fields(c, inner);
    EMember& M = E->table_host[i];
    std::memset(&M, 0, sizeof(M));
    M.g = c->geo;
    M.t0 = t0;
    M.nt = ceil_div(c->geo.vh, tb);
    M.r0 = r0;
    M.nr = ceil_div(c->geo.vh, UTB);
    t0 += M.nt;
    r0 += M.nr;
    M.gauge = c->gauge[inner];
    M.ainv = c->clov.ainv_oo[inner];
    M.aee = c->clov.a_ee[inner];
    M.gauge64 = c->gauge[LQ_F64];
    M.ainv64 = c->clov.ainv_oo[LQ_F64];
    M.aee64 = c->clov.a_ee[LQ_F64];
    M.p = f.p;
    M.q = f.q;
    M.t = f.t;
    M.xl = f.xl;
    M.r = f.r;
    M.rt = f.rt;
    M.x = f.x;
    M.bhat = f.bhat;
    M.r64 = f.r64;
    M.rn64 = f.rn64;
    M.to = f.to;
    M.st = E->st + j;
    M.k2 = c->clov.kappa * c->clov.kappa;
    LQ_CHECK(M.gauge && M.ainv && M.aee && M.gauge64 && M.ainv64 && M.aee64, LQ_ESTATE,
             "member without gauge or clover tables");
  }
  ntiles = t0;
  nutiles = r0;
  LQ_CHECK(ntiles <= E->part_rows && nutiles <= E->part_rows, LQ_EINVAL,
           "tile list longer than the partial-sum buffer");
  LQ_HIP(hipMemcpyAsync(E->table, E->table_host, sizeof(EMember) * live.size(),
                        hipMemcpyHostToDevice, E->stream));
}

template <class PO, class PV, int TB>
void launch_core(Ensemble* E, int nm, int64_t ntiles, bool finalise) {
  const dim3 g((unsigned)ntiles), b(TB), f((unsigned)nm), fb(256);
  hipStream_t s = E->stream;
  hipLaunchKernelGGL((ens_k1<PO, false, TB>), g, b, 0, s, E->table, nm);
  hipLaunchKernelGGL((ens_k2<PO, TB>), g, b, 0, s, E->table, nm, E->part);
  if (finalise) hipLaunchKernelGGL(ens_fin_alpha, f, fb, 0, s, E->table, E->part, E->due);
  hipLaunchKernelGGL((ens_k1<PO, true, TB>), g, b, 0, s, E->table, nm);
  hipLaunchKernelGGL((ens_k4<PO, PV, TB>), g, b, 0, s, E->table, nm, E->part);
  if (finalise) hipLaunchKernelGGL(ens_fin_beta, f, fb, 0, s, E->table, E->part, E->due);
  hipLaunchKernelGGL((ens_k5<PO, PV, TB>), g, b, 0, s, E->table, nm);
  LQ_HIP(hipGetLastError());
}

template <class PO, class PV>
void launch_update(Ensemble* E, int nm, int64_t nutiles) {
  const dim3 g((unsigned)std::min<int64_t>(nutiles, UGRID)), b(UTB), f((unsigned)nm), fb(256);
  hipStream_t s = E->stream;
  hipLaunchKernelGGL((ens_fold<PV>), g, b, 0, s, E->table, nm, E->due);
  hipLaunchKernelGGL((ens_res_odd<false>), g, b, 0, s, E->table, nm, E->due);
  hipLaunchKernelGGL((ens_res_even<false>), g, b, 0, s, E->table, nm, E->due, E->part);
  hipLaunchKernelGGL(ens_fin_res, f, fb, 0, s, E->table, E->part, E->due);
  hipLaunchKernelGGL((ens_res_odd<true>), g, b, 0, s, E->table, nm, E->due);
  hipLaunchKernelGGL((ens_res_even<true>), g, b, 0, s, E->table, nm, E->due, E->part);
  hipLaunchKernelGGL(ens_fin_rn, f, fb, 0, s, E->table, E->part);
  hipLaunchKernelGGL((ens_load<PO, PV>), g, b, 0, s, E->table, nm, E->due);
  LQ_HIP(hipGetLastError());
}

template <class PO, class PV>
void launch_core_tb(Ensemble* E, int tb, int nm, int64_t ntiles, bool finalise) {
  switch (tb) {
    case 64: launch_core<PO, PV, 64>(E, nm, ntiles, finalise); break;
    case 128: launch_core<PO, PV, 128>(E, nm, ntiles, finalise); break;
    default: launch_core<PO, PV, 256>(E, nm, ntiles, finalise); break;
  }
}

void core(Ensemble* E, int inner, int tb, int nm, int64_t ntiles, bool finalise) {
  switch (inner) {
    case LQ_F64: launch_core_tb<P64, P64>(E, tb, nm, ntiles, finalise); break;
    case LQ_F32: launch_core_tb<P32, P32>(E, tb, nm, ntiles, finalise); break;
    default: launch_core_tb<P16, P32>(E, tb, nm, ntiles, finalise); break;
  }
}

void update(Ensemble* E, int inner, int nm, int64_t nutiles) {
  switch (inner) {
    case LQ_F64: launch_update<P64, P64>(E, nm, nutiles); break;
    case LQ_F32: launch_update<P32, P32>(E, nm, nutiles); break;
    default: launch_update<P16, P32>(E, nm, nutiles); break;
  }
}

void sync_callers(Ensemble* E) {
  for (lq_ctx* c : E->mem) {
    if (c->stream) LQ_HIP(hipStreamSynchronize(c->stream));
    else LQ_HIP(hipDeviceSynchronize());
  }
}

// Members' kernels go to the batch's stream while the batch runs.
struct StreamSwap {
  Ensemble* E;
  std::vector<hipStream_t> saved;
  explicit StreamSwap(Ensemble* e) : E(e) {
    for (lq_ctx* c : E->mem) {
      saved.push_back(c->cur);
      c->cur = E->stream;
    }
  }
  ~StreamSwap() {
    for (size_t j = 0; j < E->mem.size(); ++j) E->mem[j]->cur = saved[j];
  }
};

void check_members(Ensemble* E, int inner) {
  LQ_CHECK(inner == LQ_F64 || inner == LQ_F32 || inner == LQ_F16, LQ_EINVAL,
           "bad inner precision");
  for (lq_ctx* c : E->mem) {
    LQ_CHECK(c->have_gauge, LQ_ESTATE, "a member has no gauge field");
    LQ_CHECK(c->clov.valid, LQ_ESTATE, "a member has no clover term (lq_set_clover)");
  }
}

}  // namespace

Ensemble* ensemble_create(lq_ctx* const* members, int n) {
  LQ_CHECK(members && n >= 1 && n <= ENS_MAX, LQ_EINVAL, "1..64 member contexts");
  for (int i = 0; i < n; ++i) {
    LQ_CHECK(members[i], LQ_EINVAL, "null member context");
    for (int k = 0; k < i; ++k)
      LQ_CHECK(members[k] != members[i], LQ_EINVAL, "a context appears twice in the batch");
  }
  Ensemble* E = new Ensemble();
  try {
    E->mem.assign(members, members + n);
    LQ_HIP(hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&E->table), sizeof(EMember) * n));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&E->table_host), sizeof(EMember) * n,
                         hipHostMallocDefault));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&E->st), sizeof(EState) * n));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&E->st_host), sizeof(EState) * n,
                         hipHostMallocDefault));
    int64_t rows = 0;
    for (lq_ctx* c : E->mem) rows += ceil_div(c->geo.vh, TILE_CHOICES[0]);
    E->part_rows = rows;
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&E->part), sizeof(double) * 2 * rows));
    LQ_HIP(hipMalloc(reinterpret_cast<void**>(&E->due), sizeof(Mask)));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&E->due_host), sizeof(Mask),
                         hipHostMallocDefault));
  } catch (...) {
    ensemble_destroy(E);
    throw;
  }
  return E;
}

void ensemble_destroy(Ensemble* E) {
  if (!E) return;
  if (E->stream) (void)hipStreamSynchronize(E->stream);
  if (E->graph) (void)hipGraphExecDestroy(E->graph);
  if (E->table) (void)hipFree(E->table);
  if (E->table_host) (void)hipHostFree(E->table_host);
  if (E->st) (void)hipFree(E->st);
  if (E->st_host) (void)hipHostFree(E->st_host);
  if (E->part) (void)hipFree(E->part);
  if (E->due) (void)hipFree(E->due);
  if (E->due_host) (void)hipHostFree(E->due_host);
  if (E->stream) (void)hipStreamDestroy(E->stream);
  delete E;
}

// Tile choice for the inner precision: the in-memory cache, else the cache
// file, else a measurement of every candidate (written back to the file).
void ensemble_tune(Ensemble* E, int inner, const char* cache_path, lq_ensemble_report* rep) {
  check_members(E, inner);
  const std::string key = tune_key(E, inner);
  TuneEntry t;
  auto it = E->tuned.find(key);
  if (it != E->tuned.end()) {
    t = it->second;
  } else {
    bool have = false;
    if (cache_path && *cache_path) {
      const auto all = read_cache(cache_path);
      auto c = all.find(key);
      if (c != all.end() && parse_entry(c->second, t)) {
        t.from_cache = true;
        have = true;
      }
    }
    if (!have) {
      sync_callers(E);
      StreamSwap sw(E);
      const int nm = (int)E->mem.size();
      std::vector<int> all(nm);
      for (int j = 0; j < nm; ++j) all[j] = j;
      // iterate with alpha = beta = 0 on the work fields (the values do not
      // change the kernels' work); the solve initialises everything again
      for (int j = 0; j < nm; ++j) {
        EState& s = E->st_host[j];
        std::memset(&s, 0, sizeof(EState));
        s.cg.active = 1;
      }
      LQ_HIP(hipMemcpyAsync(E->st, E->st_host, sizeof(EState) * nm, hipMemcpyHostToDevice,
                            E->stream));
      hipEvent_t e0, e1;
      LQ_HIP(hipEventCreate(&e0));
      LQ_HIP(hipEventCreate(&e1));
      double best = 1e300;
      constexpr int REPS = 6;
      try {
        for (int c = 0; c < 3; ++c) {
          const int tb = TILE_CHOICES[c];
          int64_t nt = 0, nu = 0;
          build_table(E, inner, tb, all, nt, nu);
          core(E, inner, tb, nm, nt, false);  // warm-up
          LQ_HIP(hipEventRecord(e0, E->stream));
          for (int r = 0; r < REPS; ++r) core(E, inner, tb, nm, nt, false);
          LQ_HIP(hipEventRecord(e1, E->stream));
          LQ_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          LQ_HIP(hipEventElapsedTime(&ms, e0, e1));
          t.ms[c] = ms / REPS;
          if (t.ms[c] < best) {
            best = t.ms[c];
            t.tile = tb;
          }
        }
      } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (cache_path && *cache_path) write_cache(cache_path, key, t);
    }
    E->tuned[key] = t;
  }
  if (rep) {
    rep->tile_sites = t.tile;
    rep->tile_from_cache = t.from_cache ? 1 : 0;
    for (int c = 0; c < 3; ++c) rep->tune_ms[c] = t.ms[c];
  }
}

void ensemble_solve(Ensemble* E, void* const* dev_x, const void* const* dev_b,
                    const double* kappa, const double* csw, double tol,
                    const lq_solver_params* prm, lq_solve_report* reports,
                    lq_ensemble_report* rep) {
  lq_solver_params p{};
  if (prm) p = *prm;
  LQ_CHECK(p.solver == LQ_CGNR, LQ_EINVAL, "the uneven batch runs CG on the normal equations");
  LQ_CHECK(!p.batched && !p.profile, LQ_EINVAL,
           "batched and profile do not apply to the uneven batch");
  LQ_CHECK(!p.fault_inject || p.inner_prec != LQ_F64, LQ_EINVAL,
           "fault_inject needs a mixed-precision inner iteration");
  const int inner = p.inner_prec;
  const int nm = (int)E->mem.size();
  for (int j = 0; j < nm; ++j) {
    LQ_CHECK(dev_x[j] && dev_b[j] && dev_x[j] != dev_b[j], LQ_EINVAL,
             "null or aliased member fields");
    LQ_CHECK(kappa[j] > 0.0 && kappa[j] < 0.25 && csw[j] >= 0.0, LQ_EINVAL, "bad kappa or csw");
  }
  const int maxiter = p.maxiter > 0 ? p.maxiter : 20000;
  const double delta = inner == LQ_F64 ? 0.0 : (p.delta > 0.0 ? p.delta : 0.1);
  const int check_every = p.check_every > 0 ? p.check_every : 8;
  const bool use_graph = p.use_graph >= 0;
  sync_callers(E);
  auto t_start = std::chrono::steady_clock::now();
  StreamSwap sw(E);
  for (int j = 0; j < nm; ++j) {
    lq_ctx* c = E->mem[j];
    LQ_CHECK(c->have_gauge, LQ_ESTATE, "a member has no gauge field");
    if (!c->clov.valid || c->clov.kappa != kappa[j] || c->clov.csw != csw[j])
      build_clover(c, kappa[j], csw[j]);
  }
  lq_ensemble_report er{};
  ensemble_tune(E, inner, nullptr, &er);
  const int tb = er.tile_sites;
  double kb[LQ_NK];
  iteration_bytes(inner, kb);
  const double site_iter = kb[0] + kb[1] + kb[2] + kb[3] + kb[4];
  // update stage per site: fold (x r/w, xl r/w), two FP64 Schur steps, load
  const double Sv = spinor_site_bytes(inner == LQ_F64 ? LQ_F64 : LQ_F32);
  const double S64 = spinor_site_bytes(LQ_F64), So = spinor_site_bytes(inner);
  const double site_update = 2 * S64 + 2 * Sv +
                             2 * (16 * link_site_bytes(LQ_F64) + 6 * S64 +
                                  2 * clover_site_bytes(LQ_F64)) +
                             2 * S64 + 2 * Sv + 2 * So;

  std::vector<double> b2(nm, 0.0), bhat_norm(nm, 0.0), bytes0(nm, 0.0);
  std::vector<SolveTally> tally(nm);
  std::vector<int> live;
  for (int j = 0; j < nm; ++j) {
    lq_ctx* c = E->mem[j];
    bytes0[j] = c->bytes;
    b2[j] = solve_begin(c, dev_x[j], dev_b[j], &bhat_norm[j]);
    tally[j].dslash += 1;
    EState& s = E->st_host[j];
    std::memset(&s, 0, sizeof(EState));
    s.done = b2[j] == 0.0 ? E_CONV : E_RUN;
    s.ru = s.done == E_RUN ? 1 : 0;
    s.updates = -1;  // the first pass of the update stage forms the initial residuals
    s.stall_iters = inner == LQ_F64 ? 0 : STALL_ITERS;
    // tests: with fault_inject the members whose index is even withhold
    // every inner correction from the FP64 solution (the initial residual
    // is formed normally), so they must stagnate and fall back
    s.withhold = (p.fault_inject && j % 2 == 0) ? 1 : 0;
    s.ref_rt2 = INFINITY;
    const double target = 0.5 * tol * bhat_norm[j];
    s.cg.target2 = target * target;
    s.cg.delta2 = delta * delta;
    s.cg.maxiter = maxiter;
    s.cg.reason = R_RUN;
    if (s.done == E_RUN) {
      live.push_back(j);
      const SolveFields f = solve_fields(c, inner);
      LQ_HIP(hipMemsetAsync(f.xl, 0, parity_field_bytes(c->geo.nblk, inner == LQ_F64 ? LQ_F64
                                                                                   : LQ_F32),
                            E->stream));
    }
  }
  LQ_HIP(hipMemcpyAsync(E->st, E->st_host, sizeof(EState) * nm, hipMemcpyHostToDevice,
                        E->stream));
  int captures = 0, replays = 0;
  if (!live.empty()) {
    int64_t nt = 0, nu = 0;
    build_table(E, inner, tb, live, nt, nu);
    int tbl_n = (int)live.size();
    int64_t tbl_tiles = nt;
    *E->due_host = tbl_n == 64 ? ~Mask(0) : (Mask(1) << tbl_n) - 1;  // every member
    LQ_HIP(hipMemcpyAsync(E->due, E->due_host, sizeof(Mask), hipMemcpyHostToDevice, E->stream));
    update(E, inner, tbl_n, nu);  // initial residuals; starts the iteration
    const int max_chunks = maxiter / check_every + 4;
    for (int chunk = 0; chunk < max_chunks; ++chunk) {
      if (use_graph) {
        std::ostringstream k;
        k << tb << "/" << check_every << "/" << inner;
        for (int i = 0; i < tbl_n; ++i) k << "," << live[i];
        if (!E->graph || E->graph_key != k.str()) {
          if (E->graph) {
            (void)hipGraphExecDestroy(E->graph);
            E->graph = nullptr;
            E->graph_key.clear();
          }
          hipGraph_t gr = nullptr;
          LQ_HIP(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
          try {
            for (int i = 0; i < check_every; ++i) {
              core(E, inner, tb, tbl_n, tbl_tiles, true);
              update(E, inner, tbl_n, nu);
            }
          } catch (...) {
            (void)hipStreamEndCapture(E->stream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
          }
          LQ_HIP(hipStreamEndCapture(E->stream, &gr));
          hipError_t e = hipGraphInstantiate(&E->graph, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          LQ_HIP(e);
          E->graph_key = k.str();
          ++captures;
        }
        LQ_HIP(hipGraphLaunch(E->graph, E->stream));
      } else {
        for (int i = 0; i < check_every; ++i) {
          core(E, inner, tb, tbl_n, tbl_tiles, true);
          update(E, inner, tbl_n, nu);
        }
      }
      ++replays;
      LQ_HIP(hipMemcpyAsync(E->st_host, E->st, sizeof(EState) * nm, hipMemcpyDeviceToHost,
                            E->stream));
      LQ_HIP(hipStreamSynchronize(E->stream));
      std::vector<int> still;
      int64_t still_tiles = 0;
      for (int i = 0; i < tbl_n; ++i)
        if (E->st_host[live[i]].done == E_RUN) {
          still.push_back(live[i]);
          still_tiles += ceil_div(E->mem[live[i]]->geo.vh, tb);
        }
      if (still.empty()) break;
      if (still_tiles * 4 <= tbl_tiles * 3) {  // drop the finished members
        live = still;
        tbl_n = (int)live.size();
        build_table(E, inner, tb, live, nt, nu);
        tbl_tiles = nt;
      }
    }
  }
  // finish every member: fallback or refinement on its own, reconstruction
  LQ_HIP(hipMemcpyAsync(E->st_host, E->st, sizeof(EState) * nm, hipMemcpyDeviceToHost,
                        E->stream));
  LQ_HIP(hipStreamSynchronize(E->stream));
  std::string msg;
  lq_status worst = LQ_OK;
  double total_bytes = 0.0;
  int max_iter = 0;
  for (int j = 0; j < nm; ++j) {
    lq_ctx* c = E->mem[j];
    const EState& s = E->st_host[j];
    SolveTally& t = tally[j];
    const int iters = s.cg.iter;
    const int ups = std::max(0, s.updates);
    t.iterations += iters;
    t.reliable += ups;
    t.dslash += 4 * iters + 4 * (ups + 1);
    max_iter = std::max(max_iter, iters);
    const double batch_bytes =
        (double)c->geo.vh * (site_iter * iters + site_update * (ups + 1));
    double res2 = 0.0, schur2 = 0.0;
    bool ok = true;
    if (b2[j] > 0.0) {
      bool conv = s.done == E_CONV;
      const int left = std::max(1, maxiter - iters);
      if (s.done == E_FALLBACK || s.done == E_RUN) {
        t.fallback = 1;
        conv = solve_more(c, LQ_F64, 0.5 * tol * bhat_norm[j], left, check_every, use_graph, t);
      }
      res2 = solve_end(c, &schur2, t);
      ok = res2 <= tol * tol * b2[j];
      double frac = 0.25;
      for (int round = 0; round < 3 && !ok && conv; ++round, frac *= 0.5) {
        conv = solve_more(c, inner, frac * tol * bhat_norm[j], std::max(1, maxiter - t.iterations),
                          check_every, use_graph, t);
        res2 = solve_end(c, &schur2, t);
        ok = res2 <= tol * tol * b2[j];
      }
    }
    const double member_bytes = c->bytes - bytes0[j] + batch_bytes;
    total_bytes += member_bytes;
    if (reports) {
      lq_solve_report& r = reports[j];
      std::memset(&r, 0, sizeof(r));
      r.iterations = t.iterations;
      r.reliable_updates = t.reliable;
      r.fallback = t.fallback;
      r.dslash_calls = t.dslash;
      r.true_residual = b2[j] > 0.0 ? std::sqrt(res2 / b2[j]) : 0.0;
      r.schur_residual = bhat_norm[j] > 0.0 ? std::sqrt(schur2) / bhat_norm[j] : 0.0;
      r.bytes = member_bytes;
      for (int k = 0; k < LQ_NK; ++k) r.kernel_bytes[k] = kb[k] * (double)c->geo.vh;
    }
    if (!ok && worst == LQ_OK) {
      worst = LQ_ENOCONV;
      msg = "member " + std::to_string(j) + " did not reach the tolerance";
    }
  }
  LQ_HIP(hipStreamSynchronize(E->stream));
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (reports)
    for (int j = 0; j < nm; ++j) reports[j].seconds = secs;
  if (rep) {
    *rep = er;
    rep->graph_captures = captures;
    rep->replays = replays;
    rep->iterations = max_iter;
    rep->seconds = secs;
    rep->bytes = total_bytes;
  }
  if (worst != LQ_OK) throw Error(worst, msg);
}

}  // namespace lq
