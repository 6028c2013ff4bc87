// Solvers of M x = b through the even-odd Schur system (include/lq.h).
//
// The plain method is CG on the normal equations of Mhat in FP64.  Mixed
// precision follows the paper's iterative-refinement idea (section 5): the
// iteration runs with FP32 or FP16 fields while FP64 holds the solution;
// whenever the inner residual has dropped by a factor delta since the last
// update (a "reliable update"), the inner correction is added to the FP64
// solution, the Schur residual is recomputed in FP64 from the operator, and
// the inner residuals are replaced by it.  The solve ends on the FP64 true
// residual of the full system, after reconstructing the odd sites.
//
// Fallback: a NaN/breakdown in the inner iteration, or five consecutive
// reliable updates without halving the FP64 residual, hands the solve to
// the plain FP64 iteration, started from the current FP64 solution.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "bicgstab_kernels.h"
#include "blockcg_kernels.h"
#include "mrhs_kernels.h"
#include "small_dense.h"
#include "solver_kernels.h"

namespace lq {

struct Work {
  int64_t nblk = 0;
  // FP64 fields
  void* b_own = nullptr;   // full-lattice buffers for host-array solves
  void* x_own = nullptr;
  void* b = nullptr;       // current right-hand side: even half then odd half (FP64)
  void* x = nullptr;       // current solution (FP64, full lattice)
  void* bhat = nullptr;    // even
  void* r64 = nullptr;     // even: bhat - Mhat x
  void* rn64 = nullptr;    // even: Mhat^+ r64
  void* te = nullptr;      // even scratch
  void* to = nullptr;      // odd scratch
  void* to2 = nullptr;     // odd scratch
  // inner-iteration fields per inner precision (index = operator precision)
  void* p[3] = {nullptr, nullptr, nullptr};
  void* q[3] = {nullptr, nullptr, nullptr};
  void* t[3] = {nullptr, nullptr, nullptr};
  void* xl[3] = {nullptr, nullptr, nullptr};  // vector precision: F64 for F64, F32 otherwise
  void* r[3] = {nullptr, nullptr, nullptr};
  void* rt[3] = {nullptr, nullptr, nullptr};
  CGState* st = nullptr;       // device
  CGState* st_host = nullptr;  // pinned
  // BiCGStab extras (operator precision): s and M s
  void* bs[3] = {nullptr, nullptr, nullptr};
  void* bt[3] = {nullptr, nullptr, nullptr};
  BiState* bst = nullptr;       // device
  BiState* bst_host = nullptr;  // pinned
  hipGraphExec_t bgraph[3] = {nullptr, nullptr, nullptr};
  int bgraph_iters[3] = {0, 0, 0};
  double bgraph_k2[3] = {0, 0, 0};
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  int graph_iters[3] = {0, 0, 0};
  double graph_k2[3] = {0, 0, 0};
  // learned-preconditioner solvers: FP32 one-parity fields
  std::vector<void*> nv, nz, nx;  // Krylov basis, preconditioned basis, work
  void* vptr = nullptr;           // device copy of the basis pointers
  int vptr_n = 0;
  double* mpart = nullptr;        // Gram-Schmidt partials, results, coefficients
  double* mres = nullptr;
  double* mcoef = nullptr;
};

namespace {

void* dalloc(size_t bytes) {
  void* p = nullptr;
  LQ_HIP(hipMalloc(&p, bytes));
  return p;
}

int vec_prec(int op_prec) { return op_prec == LQ_F64 ? LQ_F64 : LQ_F32; }

Work* work(lq_ctx* ctx, int inner) {
  if (!ctx->work) {
    Work* w = new Work();
    ctx->work = w;
    w->nblk = ctx->geo.nblk;
    const size_t f64 = parity_field_bytes(w->nblk, LQ_F64);
    w->b_own = dalloc(2 * f64);
    w->x_own = dalloc(2 * f64);
    w->bhat = dalloc(f64);
    w->r64 = dalloc(f64);
    w->rn64 = dalloc(f64);
    w->te = dalloc(f64);
    w->to = dalloc(f64);
    w->to2 = dalloc(f64);
    w->st = reinterpret_cast<CGState*>(dalloc(sizeof(CGState)));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->st_host), sizeof(CGState), hipHostMallocDefault));
  }
  Work* w = ctx->work;
  if (!w->p[inner]) {
    const size_t fo = parity_field_bytes(w->nblk, inner);
    const size_t fv = parity_field_bytes(w->nblk, vec_prec(inner));
    w->p[inner] = dalloc(fo);
    w->q[inner] = dalloc(fo);
    w->t[inner] = dalloc(fo);
    w->xl[inner] = dalloc(fv);
    w->r[inner] = dalloc(fv);
    w->rt[inner] = dalloc(fv);
  }
  return w;
}

template <class P>
Field<P> F(void* p, int64_t nblk) {
  return field_at<P>(p, nblk);
}

char* odd_half(void* full, int64_t nblk) {
  return reinterpret_cast<char*>(full) + parity_field_bytes(nblk, LQ_F64);
}

template <class PX, class PY, class PO>
void axpby(lq_ctx* ctx, void* out, double a, const void* x, double b, const void* y) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * (spinor_site_bytes(PX::id) + spinor_site_bytes(PY::id) +
                                spinor_site_bytes(PO::id));
  hipLaunchKernelGGL((axpby_kernel<PX, PY, PO>), dim3(grid_for(g.vh, SBLK)), dim3(SBLK), 0,
                     ctx->cur, g, F<PO>(out, g.nblk), a, F<PX>(const_cast<void*>(x), g.nblk), b,
                     F<PY>(const_cast<void*>(y), g.nblk));
  LQ_HIP(hipGetLastError());
}
void axpby64(lq_ctx* ctx, void* out, double a, const void* x, double b, const void* y) {
  axpby<P64, P64, P64>(ctx, out, a, x, b, y);
}

template <class PO>
void zero(lq_ctx* ctx, void* out) {
  const Geo& g = ctx->geo;
  ctx->bytes += (double)g.vh * spinor_site_bytes(PO::id);
  hipLaunchKernelGGL(zero_kernel<PO>, dim3(grid_for(g.vh, SBLK)), dim3(SBLK), 0, ctx->cur, g,
                     F<PO>(out, g.nblk));
  LQ_HIP(hipGetLastError());
}

double nrm2(lq_ctx* ctx, const void* a) {
  double v = 0;
  norm2(ctx, &v, a, LQ_F64);
  return v;
}

// ------------------------------------------------------------ CG iteration
// Algorithmic bytes per site of each kernel of one iteration (operator
// precision po, vector precision pv).
void iteration_site_bytes(int po, int pv, double out[LQ_NK]) {
  const double L = link_site_bytes(po), S = spinor_site_bytes(po), C = clover_site_bytes(po);
  const double Sv = spinor_site_bytes(pv);
  out[LQ_K_HOP_OE] = 8 * L + 2 * S + C;
  out[LQ_K_HOP_EO] = 8 * L + 3 * S + C;
  out[LQ_K_HOPD_OE] = 8 * L + 2 * S + C;
  out[LQ_K_UPDATE] = 8 * L + 3 * S + C + 6 * Sv;
  out[LQ_K_PUPDATE] = Sv + 2 * S;
}

// Per-kernel HIP-event timing of the iteration kernels (profile mode).
struct Prof {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double ms[LQ_NK] = {0, 0, 0, 0, 0};
  int calls[LQ_NK] = {0, 0, 0, 0, 0};
  hipStream_t s = nullptr;
  void begin() { LQ_HIP(hipEventRecord(e0, s)); }
  void end(int k) {
    LQ_HIP(hipEventRecord(e1, s));
    LQ_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    LQ_HIP(hipEventElapsedTime(&t, e0, e1));
    ms[k] += t;
    calls[k] += 1;
  }
};

template <class PO, class PV>
void launch_iteration(lq_ctx* ctx, Work* w, int ip, double k2d, Prof* pf = nullptr) {
  const Geo& g = ctx->geo;
  const int64_t nb = g.nblk;
  const dim3 grid(grid_for(g.vh, SBLK)), blk(SBLK);
  using S = typename PO::S;
  const S* gp = reinterpret_cast<const S*>(ctx->gauge[PO::id]);
  const S* ai = reinterpret_cast<const S*>(ctx->clov.ainv_oo[PO::id]);
  const S* ae = reinterpret_cast<const S*>(ctx->clov.a_ee[PO::id]);
  const typename PO::R k2 = (typename PO::R)k2d;
  RedBuf rb = red_buf(ctx);
  Field<PO> p = F<PO>(w->p[ip], nb), q = F<PO>(w->q[ip], nb), t = F<PO>(w->t[ip], nb);
  Field<PV> x = F<PV>(w->xl[ip], nb), r = F<PV>(w->r[ip], nb), rt = F<PV>(w->rt[ip], nb);
  if (pf) pf->begin();
  hipLaunchKernelGGL((cg_k1<PO, false>), grid, blk, 0, ctx->cur, g, &w->st->active, t, p, gp, ai);
  if (pf) pf->end(LQ_K_HOP_OE), pf->begin();
  hipLaunchKernelGGL((cg_k2<PO>), grid, blk, 0, ctx->cur, g, w->st, q, t, p, gp, ae, k2, rb);
  if (pf) pf->end(LQ_K_HOP_EO);
  hipLaunchKernelGGL((finalize_kernel<1, FinAlpha>), dim3(1), dim3(256), 0, ctx->cur, rb,
                     (int)grid.x, FinAlpha{w->st});
  if (pf) pf->begin();
  hipLaunchKernelGGL((cg_k1<PO, true>), grid, blk, 0, ctx->cur, g, &w->st->active, t, q, gp, ai);
  if (pf) pf->end(LQ_K_HOPD_OE), pf->begin();
  hipLaunchKernelGGL((cg_k4<PO, PV>), grid, blk, 0, ctx->cur, g, w->st, t, q, p, x, r, rt, gp,
                     ae, k2, rb);
  if (pf) pf->end(LQ_K_UPDATE);
  hipLaunchKernelGGL((finalize_kernel<2, FinBeta>), dim3(1), dim3(256), 0, ctx->cur, rb,
                     (int)grid.x, FinBeta{w->st});
  if (pf) pf->begin();
  hipLaunchKernelGGL((cg_k5<PO, PV>), grid, blk, 0, ctx->cur, g, w->st, p, r);
  if (pf) pf->end(LQ_K_PUPDATE);
  LQ_HIP(hipGetLastError());
}

template <class PO, class PV>
void run_iterations(lq_ctx* ctx, Work* w, int ip, double k2, int n, bool use_graph,
                    Prof* pf) {
  if (pf) {
    // one iteration at a time, so that no timed launch is a no-op
    launch_iteration<PO, PV>(ctx, w, ip, k2, pf);
    return;
  }
  if (!use_graph) {
    for (int i = 0; i < n; ++i) launch_iteration<PO, PV>(ctx, w, ip, k2);
    return;
  }
  if (!w->graph[ip] || w->graph_iters[ip] != n || w->graph_k2[ip] != k2) {
    if (w->graph[ip]) {
      (void)hipGraphExecDestroy(w->graph[ip]);
      w->graph[ip] = nullptr;
    }
    hipGraph_t gr = nullptr;
    LQ_HIP(hipStreamBeginCapture(ctx->cur, hipStreamCaptureModeThreadLocal));
    try {
      for (int i = 0; i < n; ++i) launch_iteration<PO, PV>(ctx, w, ip, k2);
    } catch (...) {
      (void)hipStreamEndCapture(ctx->cur, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    LQ_HIP(hipStreamEndCapture(ctx->cur, &gr));
    hipError_t e = hipGraphInstantiate(&w->graph[ip], gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    LQ_HIP(e);
    w->graph_iters[ip] = n;
    w->graph_k2[ip] = k2;
  }
  LQ_HIP(hipGraphLaunch(w->graph[ip], ctx->cur));
}

struct SolveStats {
  int iterations = 0;
  int reliable = 0;
  int fallback = 0;
  int dslash = 0;
};

// Schur residual r64 = bhat - Mhat x_e (FP64); returns |r64|^2.
double schur_residual(lq_ctx* ctx, Work* w, SolveStats& ss) {
  schur(ctx, w->te, w->x, w->to, 0, LQ_F64);
  axpby64(ctx, w->r64, 1.0, w->bhat, -1.0, w->te);
  ss.dslash += 2;
  return nrm2(ctx, w->r64);
}

// ||x - xref|| / ||xref|| of two full-lattice FP64 fields (even half, odd
// half), in the work space's FP64 scratch fields.
double ref_error(lq_ctx* ctx, Work* w, const void* x, const void* xref) {
  const size_t hb = parity_field_bytes(w->nblk, LQ_F64);
  const char* xc = reinterpret_cast<const char*>(x);
  const char* rc = reinterpret_cast<const char*>(xref);
  double d2 = 0.0, r2 = 0.0;
  for (int h = 0; h < 2; ++h) {
    void* tmp = h ? w->to : w->te;
    axpby64(ctx, tmp, 1.0, xc + h * hb, -1.0, rc + h * hb);
    d2 += nrm2(ctx, tmp);
    r2 += nrm2(ctx, rc + h * hb);
  }
  return r2 > 0.0 ? std::sqrt(d2 / r2) : (d2 > 0.0 ? INFINITY : 0.0);
}

// Normal residual of the restart: r = Mhat^+ r64 in the vector precision and
// rt = r64 rounded to it; returns |r|^2.  A mixed-precision iteration forms r
// with the FP32 operator from the rounded r64: r only restarts the inner
// vector, which holds FP32 accuracy anyway, for half the bytes of the FP64
// sweep.  (The FP64 residual r64 itself always comes from the FP64 operator.)
template <class PO, class PV>
double restart_residuals(lq_ctx* ctx, Work* w, int ip, SolveStats& ss) {
  ss.dslash += 2;
  if constexpr (PV::id == LQ_F64) {
    schur(ctx, w->rn64, w->r64, w->to, 1, LQ_F64);
    axpby<P64, P64, PV>(ctx, w->r[ip], 1.0, w->rn64, 0.0, w->rn64);
    axpby<P64, P64, PV>(ctx, w->rt[ip], 1.0, w->r64, 0.0, w->r64);
    return nrm2(ctx, w->rn64);
  } else {
    axpby<P64, P64, PV>(ctx, w->rt[ip], 1.0, w->r64, 0.0, w->r64);
    schur(ctx, w->r[ip], w->rt[ip], w->to, 1, LQ_F32);  // w->to: FP64 odd, holds an FP32 one
    double v = 0.0;
    norm2(ctx, &v, w->r[ip], LQ_F32);
    return v;
  }
}

template <class PO, class PV>
void load_inner_state(lq_ctx* ctx, Work* w, int ip, bool restart_p, double beta) {
  // p = r (+ beta p), r and rt already restarted
  if (restart_p)
    axpby<PV, PV, PO>(ctx, w->p[ip], 1.0, w->r[ip], 0.0, w->r[ip]);
  else
    axpby<PV, PO, PO>(ctx, w->p[ip], 1.0, w->r[ip], beta, w->p[ip]);
}

// Returns true when the Schur residual reached target; x (even half) updated.
template <class PO, class PV>
bool cg_normal(lq_ctx* ctx, Work* w, double target, double delta, int maxiter, int check_every,
               bool use_graph, int fault_inject, SolveStats& ss, bool& want_fallback,
               Prof* pf) {
  const int ip = PO::id;
  double kb[LQ_NK];
  iteration_site_bytes(PO::id, PV::id, kb);
  const double iter_bytes = (double)ctx->geo.vh * (kb[0] + kb[1] + kb[2] + kb[3] + kb[4]);
  const double last_bytes = (double)ctx->geo.vh * kb[LQ_K_PUPDATE];
  const double k2 = ctx->clov.kappa * ctx->clov.kappa;
  const double target2 = target * target;
  want_fallback = false;
  double rt2 = schur_residual(ctx, w, ss);
  if (rt2 <= target2) return true;
  double rr = restart_residuals<PO, PV>(ctx, w, ip, ss);
  zero<PV>(ctx, w->xl[ip]);
  load_inner_state<PO, PV>(ctx, w, ip, true, 0.0);
  CGState& h = *w->st_host;
  std::memset(&h, 0, sizeof(CGState));
  h.rr = rr;
  h.rt2 = rt2;
  h.rt2_max = rt2;
  h.target2 = target2;
  h.delta2 = delta * delta;
  h.active = 1;
  h.reason = R_RUN;
  h.iter = 0;
  h.maxiter = maxiter;
  LQ_HIP(hipMemcpyAsync(w->st, &h, sizeof(CGState), hipMemcpyHostToDevice, ctx->cur));
  double best_hist[6];
  int nhist = 0;
  // iteration-level stagnation: the inner residual must halve every
  // STALL_ITERS iterations, otherwise a mixed-precision solve falls back
  constexpr int STALL_ITERS = 200;
  int ref_iter = 0;
  double ref_rt2 = rt2;
  int counted = 0;
  for (;;) {
    run_iterations<PO, PV>(ctx, w, ip, k2, check_every, use_graph, pf);
    LQ_HIP(hipMemcpyAsync(&h, w->st, sizeof(CGState), hipMemcpyDeviceToHost, ctx->cur));
    LQ_HIP(hipStreamSynchronize(ctx->cur));
    // count the iterations that ran (the stopping one skips the p update)
    ctx->bytes += (h.iter - counted) * iter_bytes - (h.active ? 0.0 : last_bytes);
    counted = h.iter;
    if (h.active) {
      if (h.rt2 <= 0.25 * ref_rt2) {
        ref_iter = h.iter;
        ref_rt2 = h.rt2;
      } else if (PO::id != LQ_F64 && h.iter - ref_iter >= STALL_ITERS) {
        ss.iterations = h.iter;
        if (!fault_inject) axpby<P64, PV, P64>(ctx, w->x, 1.0, w->x, 1.0, w->xl[ip]);
        want_fallback = true;
        return false;
      }
      continue;
    }
    ss.iterations = h.iter;
    if (h.reason == R_NAN) {
      if (PO::id != LQ_F64) {
        want_fallback = true;
        return false;
      }
      throw Error(LQ_ENAN, "NaN or breakdown in the FP64 CG iteration");
    }
    // fold the inner correction into the FP64 solution
    if (!fault_inject) axpby<P64, PV, P64>(ctx, w->x, 1.0, w->x, 1.0, w->xl[ip]);
    zero<PV>(ctx, w->xl[ip]);
    rt2 = schur_residual(ctx, w, ss);
    ss.reliable += 1;
    if (!std::isfinite(rt2)) {
      if (PO::id != LQ_F64) {
        want_fallback = true;
        return false;
      }
      throw Error(LQ_ENAN, "NaN in the FP64 residual");
    }
    if (rt2 <= target2) return true;
    if (h.reason == R_MAXITER || h.iter >= maxiter) return false;
    // stagnation: five updates without halving the FP64 residual norm
    if (nhist < 6) {
      best_hist[nhist++] = rt2;
    } else {
      for (int i = 0; i < 5; ++i) best_hist[i] = best_hist[i + 1];
      best_hist[5] = rt2;
    }
    if (PO::id != LQ_F64 && nhist == 6) {
      double recent = best_hist[1];
      for (int i = 2; i < 6; ++i) recent = std::fmin(recent, best_hist[i]);
      if (recent > 0.25 * best_hist[0]) {
        want_fallback = true;
        return false;
      }
    }
    const double rr_new = restart_residuals<PO, PV>(ctx, w, ip, ss);
    // The iteration that triggered the update computed x, r and
    // beta = |r_k+1|^2 / |r_k|^2 but not p_k+1.  p continues as
    // r_new + (|r_new|^2 / |r_k|^2) p_k, with |r_k|^2 = h.rr / h.beta.
    const double beta = (h.rr > 0.0 && h.beta > 0.0) ? h.beta * rr_new / h.rr : 0.0;
    load_inner_state<PO, PV>(ctx, w, ip, false, beta);
    h.rr = rr_new;
    h.rt2 = rt2;
    h.rt2_max = rt2;
    h.active = 1;
    h.reason = R_RUN;
    if (rt2 <= 0.25 * ref_rt2) {
      ref_iter = h.iter;
      ref_rt2 = rt2;
    }
    LQ_HIP(hipMemcpyAsync(w->st, &h, sizeof(CGState), hipMemcpyHostToDevice, ctx->cur));
  }
}

bool run_cg(lq_ctx* ctx, Work* w, int inner, double target, double delta, int maxiter,
            int check_every, bool use_graph, int fault_inject, SolveStats& ss, bool& fb,
            Prof* pf) {
  switch (inner) {
    case LQ_F64:
      return cg_normal<P64, P64>(ctx, w, target, delta, maxiter, check_every, use_graph, 0, ss, fb,
                                 pf);
    case LQ_F32:
      return cg_normal<P32, P32>(ctx, w, target, delta, maxiter, check_every, use_graph,
                                 fault_inject, ss, fb, pf);
    default:
      return cg_normal<P16, P32>(ctx, w, target, delta, maxiter, check_every, use_graph,
                                 fault_inject, ss, fb, pf);
  }
}

// ------------------------------------------------------------ BiCGStab
void bicg_site_bytes(int po, int pv, double* total) {
  const double L = link_site_bytes(po), S = spinor_site_bytes(po), C = clover_site_bytes(po);
  const double Sv = spinor_site_bytes(pv);
  *total = (8 * L + 2 * S + C) * 2      // B1, B4
           + (8 * L + 3 * S + C + Sv)   // B2 (+ rh)
           + (Sv + 2 * S)               // B3
           + (8 * L + 3 * S + C)        // B5
           + (3 * Sv + 3 * S + Sv)      // B6: x r/w, p, s, tt, r write, rh
           + (Sv + 3 * S);              // B7
}

template <class PO, class PV>
void launch_bi_iteration(lq_ctx* ctx, Work* w, int ip, double k2d) {
  const Geo& g = ctx->geo;
  const int64_t nb = g.nblk;
  const dim3 grid(grid_for(g.vh, SBLK)), blk(SBLK);
  using S = typename PO::S;
  const S* gp = reinterpret_cast<const S*>(ctx->gauge[PO::id]);
  const S* ai = reinterpret_cast<const S*>(ctx->clov.ainv_oo[PO::id]);
  const S* ae = reinterpret_cast<const S*>(ctx->clov.a_ee[PO::id]);
  const typename PO::R k2 = (typename PO::R)k2d;
  RedBuf rb = red_buf(ctx);
  Field<PO> p = F<PO>(w->p[ip], nb), v = F<PO>(w->q[ip], nb), t = F<PO>(w->t[ip], nb);
  Field<PO> s = F<PO>(w->bs[ip], nb), tt = F<PO>(w->bt[ip], nb);
  Field<PV> x = F<PV>(w->xl[ip], nb), r = F<PV>(w->r[ip], nb), rh = F<PV>(w->rt[ip], nb);
  const int* act = &w->bst->active;
  hipLaunchKernelGGL((cg_k1<PO, false>), grid, blk, 0, ctx->cur, g, act, t, p, gp, ai);
  hipLaunchKernelGGL((bi_hop_eo<PO, PV, 0>), grid, blk, 0, ctx->cur, g, act, v, t, p, rh, gp, ae,
                     k2, rb);
  hipLaunchKernelGGL((finalize_kernel<3, FinBiAlpha>), dim3(1), dim3(256), 0, ctx->cur, rb,
                     (int)grid.x, FinBiAlpha{w->bst});
  hipLaunchKernelGGL((bi_s<PO, PV>), grid, blk, 0, ctx->cur, g, w->bst, s, r, v);
  hipLaunchKernelGGL((cg_k1<PO, false>), grid, blk, 0, ctx->cur, g, act, t, s, gp, ai);
  hipLaunchKernelGGL((bi_hop_eo<PO, PV, 1>), grid, blk, 0, ctx->cur, g, act, tt, t, s, rh, gp, ae,
                     k2, rb);
  hipLaunchKernelGGL((finalize_kernel<3, FinBiOmega>), dim3(1), dim3(256), 0, ctx->cur, rb,
                     (int)grid.x, FinBiOmega{w->bst});
  hipLaunchKernelGGL((bi_update<PO, PV>), grid, blk, 0, ctx->cur, g, w->bst, x, r, rh, p, s, tt,
                     rb);
  hipLaunchKernelGGL((finalize_kernel<3, FinBiRho>), dim3(1), dim3(256), 0, ctx->cur, rb,
                     (int)grid.x, FinBiRho{w->bst});
  hipLaunchKernelGGL((bi_p<PO, PV>), grid, blk, 0, ctx->cur, g, w->bst, p, r, v);
  LQ_HIP(hipGetLastError());
}

template <class PO, class PV>
void run_bi_iterations(lq_ctx* ctx, Work* w, int ip, double k2, int n, bool use_graph) {
  if (!use_graph) {
    for (int i = 0; i < n; ++i) launch_bi_iteration<PO, PV>(ctx, w, ip, k2);
    return;
  }
  if (!w->bgraph[ip] || w->bgraph_iters[ip] != n || w->bgraph_k2[ip] != k2) {
    if (w->bgraph[ip]) {
      (void)hipGraphExecDestroy(w->bgraph[ip]);
      w->bgraph[ip] = nullptr;
    }
    hipGraph_t gr = nullptr;
    LQ_HIP(hipStreamBeginCapture(ctx->cur, hipStreamCaptureModeThreadLocal));
    try {
      for (int i = 0; i < n; ++i) launch_bi_iteration<PO, PV>(ctx, w, ip, k2);
    } catch (...) {
      (void)hipStreamEndCapture(ctx->cur, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    LQ_HIP(hipStreamEndCapture(ctx->cur, &gr));
    hipError_t e = hipGraphInstantiate(&w->bgraph[ip], gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    LQ_HIP(e);
    w->bgraph_iters[ip] = n;
    w->bgraph_k2[ip] = k2;
  }
  LQ_HIP(hipGraphLaunch(w->bgraph[ip], ctx->cur));
}

// BiCGStab on Mhat x_e = bhat; restarts (with the shadow residual reset to
// the FP64 residual) at every reliable update, at a rho breakdown and when
// the recurrence reports convergence that the FP64 residual does not confirm.
template <class PO, class PV>
bool bicgstab(lq_ctx* ctx, Work* w, double target, double delta, int maxiter, int check_every,
              bool use_graph, int fault_inject, SolveStats& ss, bool& want_fallback) {
  const int ip = PO::id;
  const int64_t nb = ctx->geo.nblk;
  const double k2 = ctx->clov.kappa * ctx->clov.kappa;
  const double target2 = target * target;
  want_fallback = false;
  if (!w->bs[ip]) {
    const size_t fo = parity_field_bytes(nb, PO::id);
    w->bs[ip] = dalloc(fo);
    w->bt[ip] = dalloc(fo);
  }
  if (!w->bst) {
    w->bst = reinterpret_cast<BiState*>(dalloc(sizeof(BiState)));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->bst_host), sizeof(BiState),
                         hipHostMallocDefault));
  }
  double bytes_it = 0.0;
  bicg_site_bytes(PO::id, PV::id, &bytes_it);
  bytes_it *= (double)ctx->geo.vh;
  BiState& h = *w->bst_host;
  double hist[6];
  int nhist = 0, restarts = 0, counted = 0;
  double rt2 = schur_residual(ctx, w, ss);
  if (rt2 <= target2) return true;
  zero<PV>(ctx, w->xl[ip]);
  for (;;) {
    // (re)start from the FP64 residual: r = rh = p = r64
    axpby<P64, P64, PV>(ctx, w->r[ip], 1.0, w->r64, 0.0, w->r64);
    axpby<P64, P64, PV>(ctx, w->rt[ip], 1.0, w->r64, 0.0, w->r64);
    axpby<P64, P64, PO>(ctx, w->p[ip], 1.0, w->r64, 0.0, w->r64);
    std::memset(&h, 0, sizeof(BiState));
    h.rho[0] = rt2;
    h.rr = rt2;
    h.rr_max = rt2;
    h.rrh = rt2;
    h.target2 = target2;
    h.delta2 = delta * delta;
    h.active = 1;
    h.iter = ss.iterations;
    h.maxiter = maxiter;
    counted = h.iter;
    LQ_HIP(hipMemcpyAsync(w->bst, &h, sizeof(BiState), hipMemcpyHostToDevice, ctx->cur));
    int ref_iter = h.iter;
    double ref_rr = rt2;
    bool stalled = false;
    for (;;) {
      run_bi_iterations<PO, PV>(ctx, w, ip, k2, check_every, use_graph);
      LQ_HIP(hipMemcpyAsync(&h, w->bst, sizeof(BiState), hipMemcpyDeviceToHost, ctx->cur));
      LQ_HIP(hipStreamSynchronize(ctx->cur));
      ctx->bytes += (h.iter - counted) * bytes_it;
      counted = h.iter;
      if (!h.active) break;
      if (h.rr <= 0.25 * ref_rr) {
        ref_iter = h.iter;
        ref_rr = h.rr;
      } else if (h.iter - ref_iter >= 400) {
        stalled = true;
        break;
      }
    }
    ss.iterations = h.iter;
    if (!fault_inject) axpby<P64, PV, P64>(ctx, w->x, 1.0, w->x, 1.0, w->xl[ip]);
    zero<PV>(ctx, w->xl[ip]);
    rt2 = schur_residual(ctx, w, ss);
    ss.reliable += 1;
    if (!std::isfinite(rt2)) {
      want_fallback = true;
      return false;
    }
    if (rt2 <= target2) return true;
    if (h.reason == R_MAXITER || h.iter >= maxiter) return false;
    if (h.reason == R_NAN || stalled) restarts += 1;
    if (nhist < 6) {
      hist[nhist++] = rt2;
    } else {
      for (int i = 0; i < 5; ++i) hist[i] = hist[i + 1];
      hist[5] = rt2;
    }
    const bool no_progress = nhist == 6 && std::fmin(std::fmin(hist[1], hist[2]),
                                                     std::fmin(std::fmin(hist[3], hist[4]),
                                                               hist[5])) > 0.25 * hist[0];
    // BiCGStab stagnates on indefinite systems (a spectrum on both sides of
    // the imaginary axis), in any precision; the plain FP64 CG on the normal
    // equations takes over
    if (no_progress || restarts > 20) {
      want_fallback = true;
      return false;
    }
  }
}

// ------------------------------------------------------------ learned preconditioner
// Flexible Krylov solvers with the net N_e: FGMRES(m) on Mhat with N_e as
// right preconditioner, and flexible CG on Mhat^+ Mhat with N_e N_e^+.  The
// inner cycles run in FP32 and restart from the FP64 residual of the Schur
// system (the solution accumulates in FP64); a solve that stagnates, breaks
// down or runs out of iterations is handed to the plain mixed CG.
using cplx = std::complex<double>;

void* f32_buf(std::vector<void*>& v, size_t i, size_t bytes) {
  while (v.size() <= i) v.push_back(dalloc(bytes));
  return v[i];
}

cplx cdot32(lq_ctx* ctx, const void* a, const void* b) {
  double r[2];
  dot(ctx, r, a, b, LQ_F32);
  return {r[0], r[1]};
}

double nrm32(lq_ctx* ctx, const void* a) {
  double v = 0.0;
  norm2(ctx, &v, a, LQ_F32);
  return v;
}

// Restart bookkeeping shared by both solvers: true residual, stop, stall.
// Returns 1 = converged, 0 = continue, -1 = give up (fb set for breakdowns).
int net_restart(lq_ctx* ctx, Work* w, double target, int maxiter, double& best, int& stalls,
                SolveStats& ss, bool& fb, double& beta) {
  beta = std::sqrt(schur_residual(ctx, w, ss));
  if (!std::isfinite(beta)) {
    fb = true;
    return -1;
  }
  if (beta <= target) return 1;
  if (ss.iterations >= maxiter) return -1;
  if (beta < 0.5 * best) {
    best = beta;
    stalls = 0;
  } else if (++stalls >= 3) {
    fb = true;
    return -1;
  }
  ss.reliable += 1;
  return 0;
}

bool fgmres_net(lq_ctx* ctx, Work* w, Net* net, double target, int maxiter, int m,
                SolveStats& ss, bool& fb) {
  const size_t f32 = parity_field_bytes(ctx->geo.nblk, LQ_F32);
  std::vector<void*>& V = w->nv;
  std::vector<void*>& Z = w->nz;
  for (int i = 0; i <= m; ++i) f32_buf(V, i, f32);
  for (int i = 0; i < m; ++i) f32_buf(Z, i, f32);
  void* wv = f32_buf(w->nx, 0, f32);
  void* to32 = f32_buf(w->nx, 1, f32);
  if (w->vptr_n < m + 1) {  // device array of the basis pointers, Gram-Schmidt buffers
    for (void* q : {w->vptr, (void*)w->mpart, (void*)w->mres, (void*)w->mcoef})
      if (q) (void)hipFree(q);
    w->vptr = dalloc(sizeof(void*) * (m + 1));
    w->mpart = reinterpret_cast<double*>(dalloc(sizeof(double) * 2 * MDOT_BLOCKS_MAX * (m + 1)));
    w->mres = reinterpret_cast<double*>(dalloc(sizeof(double) * 2 * (m + 1)));
    w->mcoef = reinterpret_cast<double*>(dalloc(sizeof(double) * 2 * (m + 1)));
    w->vptr_n = m + 1;
  }
  LQ_HIP(hipMemcpyAsync(w->vptr, V.data(), sizeof(void*) * (m + 1), hipMemcpyHostToDevice,
                        ctx->cur));
  const int L = net_layers(net);
  double best = INFINITY, beta = 0.0;
  int stalls = 0;
  for (;;) {
    const int st = net_restart(ctx, w, target, maxiter, best, stalls, ss, fb, beta);
    if (st != 0) return st > 0;
    axpby<P64, P64, P32>(ctx, V[0], 1.0 / beta, w->r64, 0.0, w->r64);
    std::vector<cplx> H((size_t)(m + 1) * m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
    std::vector<double> cs(m, 1.0);
    g[0] = beta;
    // an FP32 cycle reduces the residual by at most about 1e-5 reliably
    const double inner_target = std::max(1e-4 * beta, 0.5 * target);
    int k = 0;
    while (k < m && ss.iterations < maxiter) {
      net_apply_even_fast(net, Z[k], V[k], false);
      schur(ctx, wv, Z[k], to32, 0, LQ_F32);
      ss.dslash += 2 + 2 * L;
      ss.iterations += 1;
      for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, applied twice
        std::vector<double> c(2 * (k + 1));
        multidot_f32(ctx, w->vptr, k + 1, wv, w->mpart, w->mres, c.data());
        std::vector<double> nc(2 * (k + 1));
        for (int i = 0; i <= k; ++i) {
          H[(size_t)i * m + k] += cplx(c[2 * i], c[2 * i + 1]);
          nc[2 * i] = c[2 * i];
          nc[2 * i + 1] = c[2 * i + 1];
        }
        LQ_HIP(hipMemcpyAsync(w->mcoef, nc.data(), sizeof(double) * nc.size(),
                              hipMemcpyHostToDevice, ctx->cur));
        multiaxpy_f32(ctx, w->vptr, k + 1, w->mcoef, wv);
      }
      const double hn = std::sqrt(nrm32(ctx, wv));
      if (!std::isfinite(hn)) {
        fb = true;
        return false;
      }
      H[(size_t)(k + 1) * m + k] = hn;
      if (hn > 0.0) axpby_f32(ctx, V[k + 1], 1.0 / hn, wv, 0.0, wv);
      // previous Givens rotations on column k, then the one that clears H[k+1][k]
      for (int i = 0; i < k; ++i) {
        const cplx a = H[(size_t)i * m + k], b = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + k] = -std::conj(sn[i]) * a + cs[i] * b;
      }
      const cplx a = H[(size_t)k * m + k], b = H[(size_t)(k + 1) * m + k];
      const double rho = std::sqrt(std::norm(a) + std::norm(b));
      if (std::abs(a) == 0.0) {
        cs[k] = 0.0;
        sn[k] = 1.0;
      } else {
        cs[k] = std::abs(a) / rho;
        sn[k] = (a / std::abs(a)) * std::conj(b) / rho;
      }
      H[(size_t)k * m + k] = cs[k] * a + sn[k] * b;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -std::conj(sn[k]) * g[k];
      g[k] = cs[k] * g[k];
      k += 1;
      if (std::abs(g[k]) <= inner_target || hn == 0.0) break;
    }
    // y = R^-1 g, x_e += Z y
    std::vector<cplx> y(k);
    for (int i = k - 1; i >= 0; --i) {
      cplx t = g[i];
      for (int j = i + 1; j < k; ++j) t -= H[(size_t)i * m + j] * y[j];
      y[i] = t / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) {
      if (!std::isfinite(y[i].real()) || !std::isfinite(y[i].imag())) {
        fb = true;
        return false;
      }
      caxpy_64_32(ctx, w->x, y[i].real(), y[i].imag(), Z[i]);
    }
  }
}

bool fcg_net(lq_ctx* ctx, Work* w, Net* net, double target, int maxiter, SolveStats& ss,
             bool& fb) {
  const size_t f32 = parity_field_bytes(ctx->geo.nblk, LQ_F32);
  for (int i = 0; i < 8; ++i) f32_buf(w->nx, i, f32);
  void *r = w->nx[0], *z = w->nx[1], *p = w->nx[2], *q = w->nx[3], *t = w->nx[4],
       *xl = w->nx[5], *to32 = w->nx[6], *u = w->nx[7];
  const int L = net_layers(net);
  double best = INFINITY, beta = 0.0;
  int stalls = 0;
  auto precond = [&](void* out, const void* in) {  // out = N_e N_e^+ in
    net_apply_even_fast(net, u, in, true);
    net_apply_even_fast(net, out, u, false);
    ss.dslash += 4 * L;
  };
  for (;;) {
    const int st = net_restart(ctx, w, target, maxiter, best, stalls, ss, fb, beta);
    if (st != 0) return st > 0;
    schur(ctx, w->rn64, w->r64, w->to, 1, LQ_F64);
    ss.dslash += 2;
    axpby<P64, P64, P32>(ctx, r, 1.0, w->rn64, 0.0, w->rn64);
    const double rn0 = std::sqrt(nrm32(ctx, r));
    // an FP32 cycle reduces the normal residual by about 1e-3 reliably; the
    // last cycle stops at the reduction the Schur residual still needs
    // (with a margin of 2), instead of overshooting the tolerance
    const double cycle = std::max(1e-3, 0.5 * target / beta);
    axpby_f32(ctx, xl, 0.0, r, 0.0, r);
    precond(z, r);
    axpby_f32(ctx, p, 1.0, z, 0.0, z);
    for (;;) {
      schur(ctx, t, p, to32, 0, LQ_F32);
      schur(ctx, q, t, to32, 1, LQ_F32);
      ss.dslash += 4;
      ss.iterations += 1;
      const cplx pq = cdot32(ctx, p, q), pr = cdot32(ctx, p, r);
      if (!(pq.real() > 0.0) || !std::isfinite(pq.real())) {
        fb = true;
        return false;
      }
      const cplx al = pr / pq;
      caxpy_f32(ctx, xl, al.real(), al.imag(), p);
      caxpy_f32(ctx, r, -al.real(), -al.imag(), q);
      const double rn = std::sqrt(nrm32(ctx, r));
      if (!std::isfinite(rn)) {
        fb = true;
        return false;
      }
      if (rn <= cycle * rn0 || ss.iterations >= maxiter) break;
      precond(z, r);
      // p = z + beta p with beta making p conjugate to the previous direction
      const cplx bt = -cdot32(ctx, q, z) / pq;
      caxpy_f32(ctx, z, bt.real(), bt.imag(), p);
      std::swap(w->nx[1], w->nx[2]);
      z = w->nx[1];
      p = w->nx[2];
    }
    caxpy_64_32(ctx, w->x, 1.0, 0.0, xl);
  }
}

// FGMRES with deflated restarting (krylov.hip) on Mhat with N_e on the
// right: FP32 even fields, restarts from the FP64 Schur residual.
bool fgmres_dr_net(lq_ctx* ctx, Work* w, Net* net, double target, int maxiter, int m, int k,
                   SolveStats& ss, bool& fb) {
  const size_t f32 = parity_field_bytes(ctx->geo.nblk, LQ_F32);
  void* to32 = f32_buf(w->nx, 1, f32);
  const int L = net_layers(net);
  KrylovSpace S;
  S.n = ctx->geo.nblk * SB * 12;
  S.halves = 1;
  S.vh = ctx->geo.vh;
  S.x64 = w->x;
  S.r64 = w->r64;
  S.precond = [&](void* z, const void* v) {
    net_apply_even_fast(net, z, v, false);
    ss.dslash += 2 * L;
  };
  S.op = [&](void* o, const void* z) {
    schur(ctx, o, z, to32, 0, LQ_F32);
    ss.dslash += 2;
  };
  S.residual64 = [&]() { return schur_residual(ctx, w, ss); };
  SolveTally t;
  t.iterations = ss.iterations;
  const bool conv = fgmres_dr(ctx, S, m, k, target, maxiter, t, fb);
  ss.iterations = t.iterations;
  ss.reliable += t.reliable;
  return conv;
}

bool run_inner(lq_ctx* ctx, Work* w, int solver, int inner, double target, double delta,
               int maxiter, int check_every, bool use_graph, int fault_inject, SolveStats& ss,
               bool& fb, Prof* pf, Net* net, int restart, int deflate) {
  if (solver == LQ_FGMRES_NET || solver == LQ_FCG_NET) {
    // the plain mixed CG takes over where the flexible solver gave up
    const bool conv =
        solver == LQ_FCG_NET ? fcg_net(ctx, w, net, target, maxiter, ss, fb)
        : deflate > 0        ? fgmres_dr_net(ctx, w, net, target, maxiter, restart, deflate, ss, fb)
                             : fgmres_net(ctx, w, net, target, maxiter, restart, ss, fb);
    if (conv) return true;
    fb = false;
    ss.fallback = 1;
    work(ctx, LQ_F32);
    SolveStats f_ss;
    const bool c2 = run_cg(ctx, w, LQ_F32, target, 0.1, std::max(1, maxiter - ss.iterations),
                           check_every, use_graph, 0, f_ss, fb, pf);
    ss.iterations += f_ss.iterations;
    ss.reliable += f_ss.reliable;
    ss.dslash += f_ss.dslash + 4 * f_ss.iterations;
    return c2;
  }
  if (solver == LQ_CGNR)
    return run_cg(ctx, w, inner, target, delta, maxiter, check_every, use_graph, fault_inject, ss,
                  fb, pf);
  switch (inner) {
    case LQ_F64:
      return bicgstab<P64, P64>(ctx, w, target, delta, maxiter, check_every, use_graph, 0, ss, fb);
    case LQ_F32:
      return bicgstab<P32, P32>(ctx, w, target, delta, maxiter, check_every, use_graph,
                                fault_inject, ss, fb);
    default:
      return bicgstab<P16, P32>(ctx, w, target, delta, maxiter, check_every, use_graph,
                                fault_inject, ss, fb);
  }
}

// |b|^2 of the full right-hand side w->b; bhat = b_e + kappa H_eo A_oo^-1 b_o
// (its norm in bhat_norm); x = 0.
double prepare_rhs(lq_ctx* ctx, Work* w, double& bhat_norm) {
  const int64_t nb = ctx->geo.nblk;
  const double b2 = nrm2(ctx, w->b) + nrm2(ctx, odd_half(w->b, nb));
  clover_apply(ctx, w->to, odd_half(w->b, nb), LQ_ODD, 1, LQ_F64);
  dslash(ctx, w->te, w->to, LQ_EVEN, 0, LQ_F64);
  axpby64(ctx, w->bhat, 1.0, w->b, ctx->clov.kappa, w->te);
  bhat_norm = std::sqrt(nrm2(ctx, w->bhat));
  zero<P64>(ctx, w->x);
  zero<P64>(ctx, odd_half(w->x, nb));
  return b2;
}

// x_o = A_oo^-1 (b_o + kappa H_oe x_e); returns |b - M x|^2 over both parities.
double reconstruct_and_residual(lq_ctx* ctx, Work* w, SolveStats& ss) {
  const int64_t nb = ctx->geo.nblk;
  const double kappa = ctx->clov.kappa;
  void* be = w->b;
  void* bo = odd_half(w->b, nb);
  void* xe = w->x;
  void* xo = odd_half(w->x, nb);
  dslash(ctx, w->to, xe, LQ_ODD, 0, LQ_F64);
  axpby64(ctx, w->to, 1.0, bo, kappa, w->to);
  clover_apply(ctx, xo, w->to, LQ_ODD, 1, LQ_F64);
  // r_e = b_e - A_ee x_e + kappa H_eo x_o
  clover_apply(ctx, w->te, xe, LQ_EVEN, 0, LQ_F64);
  axpby64(ctx, w->te, 1.0, be, -1.0, w->te);
  dslash(ctx, w->r64, xo, LQ_EVEN, 0, LQ_F64);
  axpby64(ctx, w->te, 1.0, w->te, kappa, w->r64);
  const double re = nrm2(ctx, w->te);
  // r_o = b_o - A_oo x_o + kappa H_oe x_e
  clover_apply(ctx, w->to, xo, LQ_ODD, 0, LQ_F64);
  axpby64(ctx, w->to, 1.0, bo, -1.0, w->to);
  dslash(ctx, w->to2, xe, LQ_ODD, 0, LQ_F64);
  axpby64(ctx, w->to, 1.0, w->to, kappa, w->to2);
  const double ro = nrm2(ctx, w->to);
  ss.dslash += 3;
  return re + ro;
}

}  // namespace

void free_work(lq_ctx* ctx) {
  Work* w = ctx->work;
  if (!w) return;
  for (void* p : {w->b_own, w->x_own, w->bhat, w->r64, w->rn64, w->te, w->to, w->to2})
    if (p) (void)hipFree(p);
  for (int i = 0; i < 3; ++i) {
    for (void* p : {w->p[i], w->q[i], w->t[i], w->xl[i], w->r[i], w->rt[i]})
      if (p) (void)hipFree(p);
    if (w->graph[i]) (void)hipGraphExecDestroy(w->graph[i]);
    for (void* p : {w->bs[i], w->bt[i]})
      if (p) (void)hipFree(p);
    if (w->bgraph[i]) (void)hipGraphExecDestroy(w->bgraph[i]);
  }
  if (w->st) (void)hipFree(w->st);
  if (w->st_host) (void)hipHostFree(w->st_host);
  if (w->bst) (void)hipFree(w->bst);
  if (w->bst_host) (void)hipHostFree(w->bst_host);
  for (auto* v : {&w->nv, &w->nz, &w->nx})
    for (void* q : *v) (void)hipFree(q);
  for (void* q : {w->vptr, (void*)w->mpart, (void*)w->mres, (void*)w->mcoef})
    if (q) (void)hipFree(q);
  delete w;
  ctx->work = nullptr;
}

// ------------------------------------------------------------ batched solve
// All right-hand sides through the multi-RHS operator (mrhs.hip).  The FP64
// part (sources, reliable updates, reconstruction, final residuals) uses the
// single-RHS FP64 kernels on each RHS's own FP64 fields.
namespace {

// Normal residual Mhat^+ r64 of a restart in FP32 (the inner vectors hold
// FP32 accuracy; the FP32 sweep moves half the bytes of the FP64 one), into
// the FP32 field w->r[LQ_F16]; returns its squared norm.
double normal_residual32(lq_ctx* ctx, Work* w, SolveStats& ss) {
  void* r32 = w->rt[LQ_F16];
  void* rn32 = w->r[LQ_F16];
  axpby<P64, P64, P32>(ctx, r32, 1.0, w->r64, 0.0, w->r64);
  schur(ctx, rn32, r32, w->to, 1, LQ_F32);  // w->to: FP64 odd, holds an FP32 one
  ss.dslash += 2;
  double v = 0.0;
  norm2(ctx, &v, rn32, LQ_F32);
  return v;
}

void solve_batched(lq_ctx* ctx, double* host_x, const double* host_b, void* dev_x,
                   const void* dev_b, int nrhs, double tol, const lq_solver_params& p,
                   lq_solve_report* report) {
  LQ_CHECK(nrhs <= MR_MAX, LQ_EINVAL, "batched solves take at most 16 right-hand sides");
  LQ_CHECK(p.solver == LQ_CGNR, LQ_EINVAL, "batched solves use CG on the normal equations");
  auto t0 = std::chrono::steady_clock::now();
  const double bytes0 = ctx->bytes;
  Work* w = work(ctx, LQ_F16);  // FP32 single fields of the restarts
  work(ctx, LQ_F64);
  MRWork* mw = mrhs_work(ctx, nrhs);
  mrhs_tables(ctx, true);  // before any graph capture
  const int64_t nb = ctx->geo.nblk;
  const int64_t nsite = ctx->V;
  const size_t hb = (size_t)nsite * 12 * 16;
  const size_t fb = 2 * parity_field_bytes(nb, LQ_F64);
  const double kappa = ctx->clov.kappa;
  const int maxiter = p.maxiter > 0 ? p.maxiter : 20000;
  // Every update event runs the FP64 single-RHS operator once per RHS still iterating, so
  // the batch triggers later than a single solve does (0.03 measured fastest at 32^3x64).
  const double delta = p.delta > 0.0 ? p.delta : 0.03;
  const int check_every = p.check_every > 0 ? p.check_every : 8;
  const bool use_graph = p.use_graph >= 0;
  void* bhat_own = w->bhat;
  std::vector<double> b2(nrhs), bhn(nrhs), res2(nrhs, 0.0), schur2(nrhs, 0.0);
  std::vector<int> done(nrhs, 0);
  SolveStats ss;
  // sources
  for (int r = 0; r < nrhs; ++r) {
    if (host_b) {
      double2* stg = reinterpret_cast<double2*>(staging(ctx, hb));
      LQ_HIP(hipMemcpyAsync(stg, host_b + (size_t)r * nsite * 24, hb, hipMemcpyHostToDevice,
                            ctx->cur));
      pack_spinor(ctx, mw->b64[r], stg, LQ_F64, LQ_FULL);
    } else {
      LQ_HIP(hipMemcpyAsync(mw->b64[r], reinterpret_cast<const char*>(dev_b) + r * fb, fb,
                            hipMemcpyDeviceToDevice, ctx->cur));
    }
    w->b = mw->b64[r];
    w->x = mw->x64[r];
    w->bhat = mw->bhat[r];
    b2[r] = nrm2(ctx, w->b) + nrm2(ctx, odd_half(w->b, nb));
    clover_apply(ctx, w->to, odd_half(w->b, nb), LQ_ODD, 1, LQ_F64);
    dslash(ctx, w->te, w->to, LQ_EVEN, 0, LQ_F64);
    axpby64(ctx, w->bhat, 1.0, w->b, kappa, w->te);
    bhn[r] = std::sqrt(nrm2(ctx, w->bhat));
    zero<P64>(ctx, w->x);
    zero<P64>(ctx, odd_half(w->x, nb));
    if (b2[r] == 0.0) done[r] = 1;
  }
  MRState& h = *mw->st_host;
  const double it_bytes = mrhs_iteration_site_bytes(nrhs) * (double)ctx->geo.vh;
  double frac = 0.5;
  bool fell_back = false;
  for (int round = 0; round < 4; ++round) {
    // (re)start every unfinished RHS from its FP64 residual
    std::memset(&h, 0, sizeof(MRState));
    h.nrhs = nrhs;
    h.delta2 = delta * delta;
    h.maxiter = maxiter;
    h.iter = ss.iterations;
    int n_on = 0;
    std::vector<double> rt2(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r) {
      mrhs_slot_from_single(ctx, mw, mw->x, LQ_F32, w->r64, r, 0.0, 0.0);
      if (done[r]) {
        mrhs_slot_from_single(ctx, mw, mw->p, LQ_F16, w->r64, r, 0.0, 0.0);
        mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r64, r, 0.0, 0.0);
        continue;
      }
      w->x = mw->x64[r];
      w->bhat = mw->bhat[r];
      rt2[r] = schur_residual(ctx, w, ss);
      const double target = frac * tol * bhn[r];
      if (rt2[r] <= target * target) {
        mrhs_slot_from_single(ctx, mw, mw->p, LQ_F16, w->r64, r, 0.0, 0.0);
        mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r64, r, 0.0, 0.0);
        continue;
      }
      const double rr = normal_residual32(ctx, w, ss);
      mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r[LQ_F16], r, 1.0, 0.0, LQ_F32);
      mrhs_slot_from_single(ctx, mw, mw->p, LQ_F16, w->r[LQ_F16], r, 1.0, 0.0, LQ_F32);
      h.on[r] = 1;
      h.rr[r] = rr;
      h.rr_max[r] = rr;
      // the inner test is on the normal residual: scale the target by the
      // ratio of the normal to the Schur residual measured here
      h.target2[r] = target * target * rr / rt2[r] * 0.25;
      ++n_on;
    }
    if (n_on > 0) {
      h.active = 1;
      mrhs_state_upload(ctx, mw);
      int counted = h.iter;
      // stagnation, as in the single-RHS solve: every iterating RHS's inner
      // residual must quarter within STALL_ITERS iterations, and its FP64
      // residual must halve within five reliable updates
      constexpr int STALL_ITERS = 200;
      std::vector<int> ref_iter(nrhs, h.iter);
      std::vector<double> ref_rr(h.rr, h.rr + nrhs);
      std::vector<std::vector<double>> hist(nrhs);
      for (int r = 0; r < nrhs; ++r)
        if (h.on[r]) hist[r].push_back(rt2[r]);
      for (;;) {
        const double bsave = ctx->bytes;
        mrhs_iterate(ctx, mw, check_every, use_graph);
        ctx->bytes = bsave;
        mrhs_state_download(ctx, mw);
        ctx->bytes += (h.iter - counted) * it_bytes;
        counted = h.iter;
        bool stalled = false;
        for (int r = 0; r < nrhs; ++r) {
          if (!h.on[r]) continue;
          if (h.rr[r] <= 0.25 * ref_rr[r]) {
            ref_rr[r] = h.rr[r];
            ref_iter[r] = h.iter;
          } else if (h.iter - ref_iter[r] >= STALL_ITERS) {
            stalled = true;
          }
        }
        if (stalled) {
          for (int r = 0; r < nrhs; ++r)
            if (h.on[r] && !p.fault_inject)
              mrhs_single_from_slot(ctx, mw, mw->x, LQ_F32, mw->x64[r], r, 1.0, 1.0);
          fell_back = true;
          break;
        }
        if (h.active) continue;
        if (h.reason == R_NAN) {
          fell_back = true;
          break;
        }
        // reliable update of every RHS still iterating
        for (int r = 0; r < nrhs; ++r) {
          if (!h.on[r]) continue;
          if (!p.fault_inject)
            mrhs_single_from_slot(ctx, mw, mw->x, LQ_F32, mw->x64[r], r, 1.0, 1.0);
          mrhs_slot_from_single(ctx, mw, mw->x, LQ_F32, w->r64, r, 0.0, 0.0);
        }
        n_on = 0;
        for (int r = 0; r < nrhs; ++r) {
          if (!h.on[r]) continue;
          w->x = mw->x64[r];
          w->bhat = mw->bhat[r];
          const double t2 = schur_residual(ctx, w, ss);
          const double target = frac * tol * bhn[r];
          if (t2 <= target * target) {
            h.on[r] = 0;
            h.alpha[r] = h.beta[r] = 0.0;
            mrhs_slot_from_single(ctx, mw, mw->p, LQ_F16, w->r64, r, 0.0, 0.0);
            mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r64, r, 0.0, 0.0);
            continue;
          }
          hist[r].push_back(t2);
          if (hist[r].size() > 6) hist[r].erase(hist[r].begin());
          if (hist[r].size() == 6 &&
              *std::min_element(hist[r].begin() + 1, hist[r].end()) > 0.25 * hist[r][0]) {
            fell_back = true;
            break;
          }
          const double rr_new = normal_residual32(ctx, w, ss);
          const double beta = (h.rr[r] > 0.0 && h.beta[r] > 0.0) ? h.beta[r] * rr_new / h.rr[r] : 0.0;
          mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r[LQ_F16], r, 1.0, 0.0, LQ_F32);
          mrhs_slot_from_single(ctx, mw, mw->p, LQ_F16, w->r[LQ_F16], r, 1.0, beta, LQ_F32);
          h.rr[r] = rr_new;
          h.rr_max[r] = rr_new;
          h.target2[r] = target * target * rr_new / t2 * 0.25;
          ref_rr[r] = rr_new;
          ref_iter[r] = h.iter;
          ++n_on;
        }
        ss.reliable += 1;
        if (fell_back || n_on == 0) break;
        if (h.reason == R_MAXITER || h.iter >= maxiter) break;
        h.active = 1;
        h.reason = R_RUN;
        mrhs_state_upload(ctx, mw);
      }
      ss.iterations = h.iter;
    }
    // finish with plain FP64 CG where the batched iteration broke down
    if (fell_back) {
      ss.fallback = 1;
      for (int r = 0; r < nrhs; ++r) {
        if (done[r]) continue;
        w->b = mw->b64[r];
        w->x = mw->x64[r];
        w->bhat = mw->bhat[r];
        SolveStats f_ss;
        bool fb = false;
        run_cg(ctx, w, LQ_F64, frac * tol * bhn[r], 0.0, maxiter, check_every, use_graph, 0,
               f_ss, fb, nullptr);
        ss.iterations += f_ss.iterations;
      }
    }
    // full-system check per RHS
    bool all_ok = true;
    for (int r = 0; r < nrhs; ++r) {
      if (done[r] && b2[r] == 0.0) continue;
      w->b = mw->b64[r];
      w->x = mw->x64[r];
      w->bhat = mw->bhat[r];
      res2[r] = reconstruct_and_residual(ctx, w, ss);
      done[r] = res2[r] <= tol * tol * b2[r];
      all_ok = all_ok && done[r];
    }
    if (all_ok || fell_back || ss.iterations >= maxiter) break;
    frac *= 0.5;
  }
  ss.dslash += 4 * ss.iterations;
  // results
  for (int r = 0; r < nrhs; ++r) {
    w->x = mw->x64[r];
    w->bhat = mw->bhat[r];
    if (host_x) {
      double2* stg = reinterpret_cast<double2*>(staging(ctx, hb));
      unpack_spinor(ctx, stg, w->x, LQ_F64, LQ_FULL);
      LQ_HIP(hipMemcpyAsync(host_x + (size_t)r * nsite * 24, stg, hb, hipMemcpyDeviceToHost,
                            ctx->cur));
      LQ_HIP(hipStreamSynchronize(ctx->cur));
    } else {
      LQ_HIP(hipMemcpyAsync(reinterpret_cast<char*>(dev_x) + r * fb, w->x, fb,
                            hipMemcpyDeviceToDevice, ctx->cur));
    }
    schur2[r] = b2[r] == 0.0 ? 0.0 : schur_residual(ctx, w, ss);
  }
  LQ_HIP(hipStreamSynchronize(ctx->cur));
  w->bhat = bhat_own;
  auto t1 = std::chrono::steady_clock::now();
  bool ok = true;
  for (int r = 0; r < nrhs; ++r) {
    const bool conv = b2[r] == 0.0 || res2[r] <= tol * tol * b2[r];
    ok = ok && conv;
    if (report) {
      lq_solve_report& rep = report[r];
      std::memset(&rep, 0, sizeof(rep));
      rep.iterations = ss.iterations;
      rep.reliable_updates = ss.reliable;
      rep.fallback = ss.fallback;
      rep.dslash_calls = ss.dslash;
      rep.true_residual = b2[r] > 0.0 ? std::sqrt(res2[r] / b2[r]) : 0.0;
      rep.schur_residual = bhn[r] > 0.0 ? std::sqrt(schur2[r]) / bhn[r] : 0.0;
      rep.seconds = std::chrono::duration<double>(t1 - t0).count();
      rep.bytes = ctx->bytes - bytes0;  // whole batch
      rep.ref_error = p.dev_xref ? ref_error(ctx, w, mw->x64[r],
                                             reinterpret_cast<const char*>(p.dev_xref) + r * fb)
                                 : -1.0;
    }
  }
  if (!ok) throw Error(LQ_ENOCONV, "a right-hand side of the batch did not reach the tolerance");
}

// ------------------------------------------------------------ block CG
// Block CG (O'Leary) for the nrhs right-hand sides of a batch on the normal
// equations Mhat^+ Mhat X = Mhat^+ Bhat: one block Krylov space shared by all
// of them, in the breakdown-free form that keeps the search block P
// orthonormal and drops directions that became dependent (or belong to
// solved right-hand sides).  An iteration:
//   Q = Mhat^+ Mhat P           (the multi-RHS operator, FP16 on the matrix cores)
//   alpha = (P^H Q)^-1 P^H R,   X += P alpha,  R -= Q alpha
//   beta = -(P^H Q)^-1 Q^H R,   W = R + P beta,  P = W T
// with T = V Lambda^-1/2 from W^H W = V Lambda V^H (eigenvalues below 1e-10
// of the largest dropped).  X and R are FP32 multi-RHS fields, P and Q FP16.
// Reliable updates per right-hand side, as in the batched CG: when its
// recursive normal residual fell by delta since its last update, or below
// its target, X_j is added to the FP64 solution, the FP64 Schur residual is
// recomputed and R_j replaced by the FP32 normal residual of it (a solved
// right-hand side gets R_j = 0); Q^H R is then recomputed for beta.
}  // namespace

struct BlockWork {
  int nrhs = 0;
  void *q1 = nullptr, *qb = nullptr, *wv = nullptr;  // FP16 even, FP32 even (Q), FP32 even (W)
  double2* part = nullptr;   // [BCG_GRID][2][16][16]
  double2* res = nullptr;    // [2][16][16]
  double2* hres = nullptr;   // pinned
  float2* coef = nullptr;    // [16][16]
  float2* hcoef = nullptr;   // pinned
};

void free_block_work(lq_ctx* ctx) {
  BlockWork* bw = ctx->bwork;
  if (!bw) return;
  for (void* q : {bw->q1, bw->qb, bw->wv, (void*)bw->part, (void*)bw->res, (void*)bw->coef})
    if (q) (void)hipFree(q);
  if (bw->hres) (void)hipHostFree(bw->hres);
  if (bw->hcoef) (void)hipHostFree(bw->hcoef);
  delete bw;
  ctx->bwork = nullptr;
}

namespace {

BlockWork* block_work(lq_ctx* ctx, int nrhs) {
  BlockWork* bw = ctx->bwork;
  if (bw && bw->nrhs != nrhs) {
    free_block_work(ctx);
    bw = nullptr;
  }
  if (!bw) {
    bw = new BlockWork();
    ctx->bwork = bw;
    bw->nrhs = nrhs;
    const size_t f16 = mrhs_field_bytes(ctx->geo.nblk, LQ_F16, nrhs);
    const size_t f32 = mrhs_field_bytes(ctx->geo.nblk, LQ_F32, nrhs);
    bw->q1 = dalloc(f16);
    bw->qb = dalloc(f32);
    bw->wv = dalloc(f32);
    bw->part = reinterpret_cast<double2*>(dalloc(sizeof(double2) * BCG_GRID * 2 * 256));
    bw->res = reinterpret_cast<double2*>(dalloc(sizeof(double2) * 2 * 256));
    bw->coef = reinterpret_cast<float2*>(dalloc(sizeof(float2) * 256));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&bw->hres), sizeof(double2) * 2 * 256));
    LQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&bw->hcoef), sizeof(float2) * 256));
  }
  return bw;
}

// The launches of one block-CG stage for the padded width KM.
template <int KM>
struct BlockOps {
  lq_ctx* ctx;
  MRWork* mw;
  BlockWork* bw;
  int K;
  MField<P16> f16(void* d) const { return mfield_at<P16>(d, ctx->mr_geo.nblk, K); }
  MField<P32> f32(void* d) const { return mfield_at<P32>(d, ctx->mr_geo.nblk, K); }
  // the two K x K matrices of a Gram launch, summed, to the host: [m][i][j]
  void fetch(int nm) {
    const int nent = nm * KM * KM;
    hipLaunchKernelGGL(bcg_sum_kernel, dim3(nent), dim3(256), 0, ctx->cur, bw->part, BCG_GRID,
                       nent, bw->res);
    LQ_HIP(hipGetLastError());
    LQ_HIP(hipMemcpyAsync(bw->hres, bw->res, sizeof(double2) * nent, hipMemcpyDeviceToHost,
                          ctx->cur));
    LQ_HIP(hipStreamSynchronize(ctx->cur));
  }
  void upload(const std::vector<dense::cplx>& m) {  // K x K -> [KM][KM] FP32
    LQ_HIP(hipStreamSynchronize(ctx->cur));
    for (int i = 0; i < KM; ++i)
      for (int j = 0; j < KM; ++j) {
        const dense::cplx z = (i < K && j < K) ? m[(size_t)i * K + j] : dense::cplx(0.0);
        bw->hcoef[i * KM + j] = make_float2((float)z.real(), (float)z.imag());
      }
    LQ_HIP(hipMemcpyAsync(bw->coef, bw->hcoef, sizeof(float2) * KM * KM, hipMemcpyHostToDevice,
                          ctx->cur));
  }
  dense::cplx h(int m, int i, int j) const {
    const double2 v = bw->hres[(m * KM + i) * KM + j];
    return {v.x, v.y};
  }
  double site_bytes(double n16, double n32) const {
    return K * (n16 * spinor_site_bytes(LQ_F16) + n32 * spinor_site_bytes(LQ_F32));
  }
  void gram_pq(void* p16, void* q32, void* r32) {  // G0 = P^H Q, G1 = P^H R
    hipLaunchKernelGGL((bcg_gram_kernel<KM, P16, P32>), dim3(BCG_GRID), dim3(BCG_THREADS), 0,
                       ctx->cur, ctx->mr_geo, f16(p16), f32(q32), f32(r32), bw->part);
    LQ_HIP(hipGetLastError());
    ctx->bytes += site_bytes(1, 2) * (double)ctx->geo.vh;
    fetch(2);
  }
  void gram_qr(void* q32, void* r32) {  // G0 = Q^H Q, G1 = Q^H R
    hipLaunchKernelGGL((bcg_gram_kernel<KM, P32, P32>), dim3(BCG_GRID), dim3(BCG_THREADS), 0,
                       ctx->cur, ctx->mr_geo, f32(q32), f32(q32), f32(r32), bw->part);
    LQ_HIP(hipGetLastError());
    ctx->bytes += site_bytes(0, 2) * (double)ctx->geo.vh;
    fetch(2);
  }
  void update() {  // coef = alpha
    hipLaunchKernelGGL(bcg_update_kernel<KM>, dim3(BCG_GRID), dim3(BCG_THREADS), 0, ctx->cur,
                       ctx->mr_geo, f16(mw->p), f32(bw->qb), f32(mw->x), f32(mw->r), bw->coef,
                       bw->part);
    LQ_HIP(hipGetLastError());
    ctx->bytes += site_bytes(1, 5) * (double)ctx->geo.vh;
    fetch(2);
  }
  void dir(bool with_p) {  // coef = beta (W = R when with_p is false)
    hipLaunchKernelGGL(bcg_dir_kernel<KM>, dim3(BCG_GRID), dim3(BCG_THREADS), 0, ctx->cur,
                       ctx->mr_geo, f16(mw->p), f32(mw->r), f32(bw->wv), bw->coef, (int)with_p,
                       bw->part);
    LQ_HIP(hipGetLastError());
    ctx->bytes += site_bytes(with_p ? 1 : 0, 2) * (double)ctx->geo.vh;
    fetch(1);
  }
  void orth() {  // coef = T
    hipLaunchKernelGGL(bcg_orth_kernel<KM>, dim3(BCG_GRID), dim3(BCG_THREADS), 0, ctx->cur,
                       ctx->mr_geo, f32(bw->wv), f16(mw->p), bw->coef);
    LQ_HIP(hipGetLastError());
    ctx->bytes += site_bytes(1, 1) * (double)ctx->geo.vh;
  }
};

// T (K x K, columns past the returned rank zero) with W T orthonormal, from
// G = W^H W; rank 0 when W vanishes.
int block_orth_factor(int K, const std::vector<dense::cplx>& G, std::vector<dense::cplx>& T) {
  std::vector<dense::cplx> a = G, v;
  std::vector<double> lam;
  dense::hermitian_eig(K, a, lam, v);
  T.assign((size_t)K * K, 0.0);
  const double top = lam.empty() ? 0.0 : lam.back();
  if (!(top > 0.0) || !std::isfinite(top)) return 0;
  int rank = 0;
  for (int e = K - 1; e >= 0; --e) {  // largest first
    if (!(lam[e] > 1e-10 * top)) break;
    const double sc = 1.0 / std::sqrt(lam[e]);
    for (int i = 0; i < K; ++i) T[(size_t)i * K + rank] = v[(size_t)i * K + e] * sc;
    ++rank;
  }
  return rank;
}

// x = G_rr^-1 Y on the leading rank x rank block (rows past the rank zero);
// false if singular
bool block_solve(int K, int rank, const std::vector<dense::cplx>& G,
                 const std::vector<dense::cplx>& Y, std::vector<dense::cplx>& X) {
  X.assign((size_t)K * K, 0.0);
  for (int j = 0; j < K; ++j) {
    std::vector<dense::cplx> a((size_t)rank * rank), b(rank);
    for (int r = 0; r < rank; ++r) {
      for (int c = 0; c < rank; ++c) a[(size_t)r * rank + c] = G[(size_t)r * K + c];
      b[r] = Y[(size_t)r * K + j];
    }
    if (rank > 0 && !dense::solve(rank, a, b)) return false;
    for (int r = 0; r < rank; ++r) X[(size_t)r * K + j] = b[r];
  }
  return true;
}

template <int KM>
bool block_iterate(lq_ctx* ctx, Work* w, MRWork* mw, BlockWork* bw, int nrhs,
                   const std::vector<double>& bhn, std::vector<int>& done, double frac, double tol,
                   double delta, int maxiter, SolveStats& ss, bool& nonfinite) {
  BlockOps<KM> op{ctx, mw, bw, nrhs};
  const int K = nrhs;
  std::vector<double> rr(K, 0.0), rr_max(K, 0.0), target2(K, 0.0);
  // start: X = 0, R_j = the FP32 normal residual of the FP64 residual
  auto refresh = [&](int j, bool first) -> void {
    if (!first) mrhs_single_from_slot(ctx, mw, mw->x, LQ_F32, mw->x64[j], j, 1.0, 1.0);
    mrhs_slot_from_single(ctx, mw, mw->x, LQ_F32, w->r64, j, 0.0, 0.0);
    w->x = mw->x64[j];
    w->bhat = mw->bhat[j];
    const double t2 = schur_residual(ctx, w, ss);
    const double target = frac * tol * bhn[j];
    if (done[j] || t2 <= target * target) {
      done[j] = 1;
      mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r64, j, 0.0, 0.0);
      rr[j] = 0.0;
      return;
    }
    const double rn = normal_residual32(ctx, w, ss);
    mrhs_slot_from_single(ctx, mw, mw->r, LQ_F32, w->r[LQ_F16], j, 1.0, 0.0, LQ_F32);
    rr[j] = rr_max[j] = rn;
    target2[j] = target * target * rn / t2 * 0.25;
  };
  for (int j = 0; j < K; ++j) refresh(j, true);
  auto all_done = [&] {
    for (int j = 0; j < K; ++j)
      if (!done[j]) return false;
    return true;
  };
  if (all_done()) return true;
  // P = orth(R): W = R (beta = 0), then T from W^H W
  std::vector<dense::cplx> G((size_t)K * K), Y((size_t)K * K), Z, T;
  op.upload(std::vector<dense::cplx>((size_t)K * K, 0.0));
  op.dir(false);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) G[(size_t)i * K + j] = op.h(0, i, j);
  int rank = block_orth_factor(K, G, T);
  op.upload(T);
  op.orth();
  int stall_ref_iter = ss.iterations;
  double stall_ref = *std::max_element(rr.begin(), rr.end());
  while (rank > 0) {
    if (ss.iterations >= maxiter) return false;
    mrhs_normal(ctx, bw->qb, mw->p, mw->t, bw->q1, K);
    ss.dslash += 4;  // (mr_hop counts the sweeps' bytes)
    op.gram_pq(mw->p, bw->qb, mw->r);
    std::vector<dense::cplx> PQ((size_t)K * K), PR((size_t)K * K), alpha;
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        PQ[(size_t)i * K + j] = op.h(0, i, j);
        PR[(size_t)i * K + j] = op.h(1, i, j);
      }
    if (!block_solve(K, rank, PQ, PR, alpha)) return false;
    op.upload(alpha);
    op.update();
    ss.iterations += 1;
    std::vector<dense::cplx> QR((size_t)K * K);
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) QR[(size_t)i * K + j] = op.h(0, i, j);
    bool replaced = false;
    for (int j = 0; j < K; ++j) {
      if (done[j]) continue;
      rr[j] = op.h(1, j, j).real();
      if (!std::isfinite(rr[j])) {
        nonfinite = true;
        return false;
      }
      if (rr[j] < delta * delta * rr_max[j] || rr[j] <= target2[j]) {
        refresh(j, false);
        ss.reliable += 1;
        replaced = true;
      }
    }
    if (all_done()) return true;
    if (replaced) {  // Q^H R with the replaced columns
      op.gram_qr(bw->qb, mw->r);
      for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) QR[(size_t)i * K + j] = op.h(1, i, j);
    }
    // stagnation: the largest normal residual must quarter within 300 iterations
    const double worst = *std::max_element(rr.begin(), rr.end());
    if (worst <= 0.25 * stall_ref) {
      stall_ref = worst;
      stall_ref_iter = ss.iterations;
    } else if (ss.iterations - stall_ref_iter >= 300) {
      return false;
    }
    std::vector<dense::cplx> beta;
    for (auto& z : QR) z = -z;
    if (!block_solve(K, rank, PQ, QR, beta)) return false;
    op.upload(beta);
    op.dir(true);
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) G[(size_t)i * K + j] = op.h(0, i, j);
    rank = block_orth_factor(K, G, T);
    op.upload(T);
    op.orth();
  }
  // the search block vanished: every remaining direction is solved to
  // rounding; one last refresh decides
  for (int j = 0; j < K; ++j)
    if (!done[j]) refresh(j, false);
  return all_done();
}

void solve_block(lq_ctx* ctx, double* host_x, const double* host_b, void* dev_x,
                 const void* dev_b, int nrhs, double tol, const lq_solver_params& p,
                 lq_solve_report* report) {
  LQ_CHECK(nrhs >= 1 && nrhs <= MR_MAX, LQ_EINVAL, "block CG takes 1..16 right-hand sides");
  LQ_CHECK(p.solver == LQ_CGNR, LQ_EINVAL, "block CG runs on the normal equations (LQ_CGNR)");
  auto t0 = std::chrono::steady_clock::now();
  const double bytes0 = ctx->bytes;
  Work* w = work(ctx, LQ_F16);
  work(ctx, LQ_F64);
  MRWork* mw = mrhs_work(ctx, nrhs);
  BlockWork* bw = block_work(ctx, nrhs);
  mrhs_tables(ctx, true);
  const int64_t nb = ctx->geo.nblk;
  const int64_t nsite = ctx->V;
  const size_t hb = (size_t)nsite * 12 * 16;
  const size_t fb = 2 * parity_field_bytes(nb, LQ_F64);
  const double kappa = ctx->clov.kappa;
  const int maxiter = p.maxiter > 0 ? p.maxiter : 20000;
  const double delta = p.delta > 0.0 ? p.delta : 0.1;
  void* bhat_own = w->bhat;
  void* x_own = w->x;
  void* b_own = w->b;
  std::vector<double> b2(nrhs), bhn(nrhs), res2(nrhs, 0.0), schur2(nrhs, 0.0);
  std::vector<int> done(nrhs, 0);
  SolveStats ss;
  for (int r = 0; r < nrhs; ++r) {
    if (host_b) {
      double2* stg = reinterpret_cast<double2*>(staging(ctx, hb));
      LQ_HIP(hipMemcpyAsync(stg, host_b + (size_t)r * nsite * 24, hb, hipMemcpyHostToDevice,
                            ctx->cur));
      pack_spinor(ctx, mw->b64[r], stg, LQ_F64, LQ_FULL);
    } else {
      LQ_HIP(hipMemcpyAsync(mw->b64[r], reinterpret_cast<const char*>(dev_b) + r * fb, fb,
                            hipMemcpyDeviceToDevice, ctx->cur));
    }
    w->b = mw->b64[r];
    w->x = mw->x64[r];
    w->bhat = mw->bhat[r];
    b2[r] = nrm2(ctx, w->b) + nrm2(ctx, odd_half(w->b, nb));
    clover_apply(ctx, w->to, odd_half(w->b, nb), LQ_ODD, 1, LQ_F64);
    dslash(ctx, w->te, w->to, LQ_EVEN, 0, LQ_F64);
    axpby64(ctx, w->bhat, 1.0, w->b, kappa, w->te);
    bhn[r] = std::sqrt(nrm2(ctx, w->bhat));
    zero<P64>(ctx, w->x);
    zero<P64>(ctx, odd_half(w->x, nb));
    if (b2[r] == 0.0) done[r] = 1;
  }
  double frac = 0.5;
  for (int round = 0; round < 4; ++round) {
    const int KM = nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : nrhs <= 12 ? 12 : 16;
    bool conv = false, nonfinite = false;
    switch (KM) {
      case 4: conv = block_iterate<4>(ctx, w, mw, bw, nrhs, bhn, done, frac, tol, delta, maxiter, ss, nonfinite); break;
      case 8: conv = block_iterate<8>(ctx, w, mw, bw, nrhs, bhn, done, frac, tol, delta, maxiter, ss, nonfinite); break;
      case 12: conv = block_iterate<12>(ctx, w, mw, bw, nrhs, bhn, done, frac, tol, delta, maxiter, ss, nonfinite); break;
      default: conv = block_iterate<16>(ctx, w, mw, bw, nrhs, bhn, done, frac, tol, delta, maxiter, ss, nonfinite);
    }
    if (!conv) {  // finish the unsolved right-hand sides with plain FP64 CG
      ss.fallback = 1;
      for (int r = 0; r < nrhs; ++r) {
        if (done[r]) continue;
        // the FP32 increment since the column's last reliable update, unless
        // the iteration produced non-finite values (then restart from that update)
        if (!nonfinite) mrhs_single_from_slot(ctx, mw, mw->x, LQ_F32, mw->x64[r], r, 1.0, 1.0);
        w->b = mw->b64[r];
        w->x = mw->x64[r];
        w->bhat = mw->bhat[r];
        SolveStats f_ss;
        bool fb = false;
        run_cg(ctx, w, LQ_F64, frac * tol * bhn[r], 0.0, maxiter, 8, true, 0, f_ss, fb, nullptr);
        ss.iterations += f_ss.iterations;
        ss.dslash += f_ss.dslash + 4 * f_ss.iterations;
        done[r] = 1;
      }
    }
    bool all_ok = true;
    for (int r = 0; r < nrhs; ++r) {
      if (b2[r] == 0.0) continue;
      w->b = mw->b64[r];
      w->x = mw->x64[r];
      w->bhat = mw->bhat[r];
      res2[r] = reconstruct_and_residual(ctx, w, ss);
      if (res2[r] > tol * tol * b2[r]) {
        all_ok = false;
        done[r] = 0;
      }
    }
    if (all_ok) break;
    frac *= 0.5;
  }
  for (int r = 0; r < nrhs; ++r) {
    w->b = mw->b64[r];
    w->x = mw->x64[r];
    w->bhat = mw->bhat[r];
    if (host_x) {
      double2* stg = reinterpret_cast<double2*>(staging(ctx, hb));
      unpack_spinor(ctx, stg, w->x, LQ_F64, LQ_FULL);
      LQ_HIP(hipMemcpyAsync(host_x + (size_t)r * nsite * 24, stg, hb, hipMemcpyDeviceToHost,
                            ctx->cur));
      LQ_HIP(hipStreamSynchronize(ctx->cur));
    } else {
      LQ_HIP(hipMemcpyAsync(reinterpret_cast<char*>(dev_x) + r * fb, w->x, fb,
                            hipMemcpyDeviceToDevice, ctx->cur));
    }
    schur2[r] = b2[r] == 0.0 ? 0.0 : schur_residual(ctx, w, ss);
  }
  LQ_HIP(hipStreamSynchronize(ctx->cur));
  w->bhat = bhat_own;
  w->x = x_own;
  w->b = b_own;
  auto t1 = std::chrono::steady_clock::now();
  bool ok = true;
  for (int r = 0; r < nrhs; ++r) {
    const bool conv = b2[r] == 0.0 || res2[r] <= tol * tol * b2[r];
    ok = ok && conv;
    if (report) {
      lq_solve_report& rep = report[r];
      std::memset(&rep, 0, sizeof(rep));
      rep.iterations = ss.iterations;
      rep.reliable_updates = ss.reliable;
      rep.fallback = ss.fallback;
      rep.dslash_calls = ss.dslash;
      rep.true_residual = b2[r] > 0.0 ? std::sqrt(res2[r] / b2[r]) : 0.0;
      rep.schur_residual = bhn[r] > 0.0 ? std::sqrt(schur2[r]) / bhn[r] : 0.0;
      rep.seconds = std::chrono::duration<double>(t1 - t0).count();
      rep.bytes = ctx->bytes - bytes0;
      rep.ref_error = p.dev_xref ? ref_error(ctx, w, mw->x64[r],
                                             reinterpret_cast<const char*>(p.dev_xref) + r * fb)
                                 : -1.0;
    }
  }
  if (!ok) throw Error(LQ_ENOCONV, "a right-hand side of the block solve did not reach the tolerance");
}

}  // namespace

void solve(lq_ctx* ctx, double* host_x, const double* host_b, void* dev_x, const void* dev_b,
           int nrhs, double kappa, double csw, double tol, const lq_solver_params* prm,
           lq_solve_report* report, Net* net) {
  lq_solver_params p{};
  if (prm) p = *prm;
  const bool net_solver = p.solver == LQ_FGMRES_NET || p.solver == LQ_FCG_NET;
  // the flexible solvers run their inner cycles in FP32
  const int inner = net_solver ? LQ_F32 : p.inner_prec;
  LQ_CHECK(inner == LQ_F64 || inner == LQ_F32 || inner == LQ_F16, LQ_EINVAL,
           "bad inner precision");
  LQ_CHECK(p.solver == LQ_CGNR || p.solver == LQ_BICGSTAB || net_solver, LQ_EINVAL,
           "unknown solver kind");
  LQ_CHECK(!net_solver || net, LQ_EINVAL,
           "learned-preconditioner solvers take a net (lq_solve_net)");
  LQ_CHECK(!net || net_ctx(net) == ctx, LQ_EINVAL, "the net belongs to another context");
  const int restart = p.restart > 0 ? p.restart : (p.deflate > 0 ? 70 : 32);
  LQ_CHECK(restart <= 128, LQ_EINVAL, "restart length above 128");
  LQ_CHECK(p.deflate >= 0 && (p.deflate == 0 || (p.solver == LQ_FGMRES_NET &&
                                                  p.deflate < restart && p.deflate <= 32)),
           LQ_EINVAL, "deflate: 1..min(restart-1, 32) deflated vectors, with LQ_FGMRES_NET only");
  const int maxiter = p.maxiter > 0 ? p.maxiter : 20000;
  const double delta = inner == LQ_F64 ? 0.0 : (p.delta > 0.0 ? p.delta : 0.1);
  const int check_every = p.check_every > 0 ? p.check_every : 8;
  const bool use_graph = p.use_graph >= 0;
  // everything below runs on the library stream, after the caller's work
  if (ctx->stream) LQ_HIP(hipStreamSynchronize(ctx->stream));
  else LQ_HIP(hipDeviceSynchronize());
  ctx->cur = ctx->sstream;
  if (!ctx->clov.valid || ctx->clov.kappa != kappa || ctx->clov.csw != csw)
    build_clover(ctx, kappa, csw);
  if (p.batched == 2) {
    LQ_CHECK(inner == LQ_F16, LQ_EINVAL, "block CG runs its inner iteration in FP16");
    solve_block(ctx, host_x, host_b, dev_x, dev_b, nrhs, tol, p, report);
    return;
  }
  if (p.batched && nrhs > 1) {
    LQ_CHECK(inner == LQ_F16, LQ_EINVAL, "batched solves run their inner iteration in FP16");
    solve_batched(ctx, host_x, host_b, dev_x, dev_b, nrhs, tol, p, report);
    return;
  }
  Work* w = work(ctx, inner);
  work(ctx, LQ_F64);
  const int64_t nsite = ctx->V;
  const size_t hb = (size_t)nsite * 12 * 16;
  lq_status worst = LQ_OK;
  Prof prof_obj;
  Prof* prof = nullptr;
  if (p.profile) {
    prof_obj.s = ctx->cur;
    LQ_HIP(hipEventCreate(&prof_obj.e0));
    LQ_HIP(hipEventCreate(&prof_obj.e1));
    prof = &prof_obj;
  }
  struct EvGuard {
    Prof* p;
    ~EvGuard() {
      if (p) {
        (void)hipEventDestroy(p->e0);
        (void)hipEventDestroy(p->e1);
      }
    }
  } ev_guard{prof};
  double kb[LQ_NK];
  iteration_site_bytes(inner, vec_prec(inner), kb);
  std::string msg;
  for (int rhs = 0; rhs < nrhs; ++rhs) {
    auto t0 = std::chrono::steady_clock::now();
    SolveStats ss;
    const double bytes0 = ctx->bytes;
    if (prof)
      for (int k = 0; k < LQ_NK; ++k) prof->ms[k] = 0.0, prof->calls[k] = 0;
    const int64_t nb = ctx->geo.nblk;
    const size_t fb = 2 * parity_field_bytes(nb, LQ_F64);
    if (host_b) {
      w->b = w->b_own;
      w->x = w->x_own;
      double2* stg = reinterpret_cast<double2*>(staging(ctx, hb));
      LQ_HIP(hipMemcpyAsync(stg, host_b + (size_t)rhs * nsite * 24, hb, hipMemcpyHostToDevice,
                            ctx->cur));
      pack_spinor(ctx, w->b, stg, LQ_F64, LQ_FULL);
    } else {
      w->b = const_cast<char*>(reinterpret_cast<const char*>(dev_b)) + rhs * fb;
      w->x = reinterpret_cast<char*>(dev_x) + rhs * fb;
    }
    double bhat_norm = 0.0;
    const double b2 = prepare_rhs(ctx, w, bhat_norm);
    ss.dslash += 1;
    double res2 = 0.0;
    bool ok = false;
    double frac = 0.5;
    lq_status st = LQ_OK;
    if (b2 == 0.0) {
      ok = true;
    } else {
      for (int round = 0; round < 4 && !ok; ++round) {
        bool fb = false;
        int left = maxiter - ss.iterations;
        SolveStats inner_ss;
        // once the plain FP64 CG has taken over, the tightening rounds stay with it
        const bool plain = ss.fallback;
        bool conv = plain
                        ? run_cg(ctx, w, LQ_F64, frac * tol * bhat_norm, 0.0, left, check_every,
                                 use_graph, 0, inner_ss, fb, prof)
                        : run_inner(ctx, w, p.solver, inner, frac * tol * bhat_norm, delta, left,
                                    check_every, use_graph, p.fault_inject, inner_ss, fb, prof,
                                    net, restart, p.deflate);
        ss.iterations += inner_ss.iterations;
        ss.reliable += inner_ss.reliable;
        // the flexible solvers count their own operator applications
        ss.dslash += inner_ss.dslash + (net_solver && !plain ? 0 : 4 * inner_ss.iterations);
        ss.fallback |= inner_ss.fallback;
        if (fb) {
          ss.fallback = 1;
          work(ctx, LQ_F64);
          SolveStats f_ss;
          left = maxiter - ss.iterations;
          conv = run_cg(ctx, w, LQ_F64, frac * tol * bhat_norm, 0.0, left, check_every,
                        use_graph, 0, f_ss, fb, prof);
          ss.iterations += f_ss.iterations;
          ss.reliable += f_ss.reliable;
          ss.dslash += f_ss.dslash + 4 * f_ss.iterations;
        }
        res2 = reconstruct_and_residual(ctx, w, ss);
        ok = res2 <= tol * tol * b2;
        if (!conv && !ok) break;
        frac *= 0.5;
      }
      if (!ok) st = LQ_ENOCONV;
    }
    // result to host
    if (host_x) {
      double2* stg = reinterpret_cast<double2*>(staging(ctx, hb));
      unpack_spinor(ctx, stg, w->x, LQ_F64, LQ_FULL);
      LQ_HIP(hipMemcpyAsync(host_x + (size_t)rhs * nsite * 24, stg, hb, hipMemcpyDeviceToHost,
                            ctx->cur));
    }
    const double schur2 = b2 == 0.0 ? 0.0 : schur_residual(ctx, w, ss);
    LQ_HIP(hipStreamSynchronize(ctx->cur));
    auto t1 = std::chrono::steady_clock::now();
    if (report) {
      lq_solve_report& r = report[rhs];
      r.iterations = ss.iterations;
      r.reliable_updates = ss.reliable;
      r.fallback = ss.fallback;
      r.dslash_calls = ss.dslash;
      r.true_residual = b2 > 0.0 ? std::sqrt(res2 / b2) : 0.0;
      r.schur_residual = bhat_norm > 0.0 ? std::sqrt(schur2) / bhat_norm : 0.0;
      r.seconds = std::chrono::duration<double>(t1 - t0).count();
      r.bytes = ctx->bytes - bytes0;
      r.ref_error = p.dev_xref ? ref_error(ctx, w, w->x,
                                           reinterpret_cast<const char*>(p.dev_xref) +
                                               (size_t)rhs * 2 * parity_field_bytes(w->nblk, LQ_F64))
                               : -1.0;
      for (int k = 0; k < LQ_NK; ++k) {
        r.kernel_bytes[k] = kb[k] * (double)ctx->geo.vh;
        r.kernel_ms[k] = prof ? prof->ms[k] : 0.0;
        r.kernel_calls[k] = prof ? prof->calls[k] : 0;
      }
    }
    if (st != LQ_OK && worst == LQ_OK) {
      worst = st;
      msg = "right-hand side " + std::to_string(rhs) + " did not reach the tolerance";
    }
  }
  if (worst != LQ_OK) throw Error(worst, msg);
}


// ------------------------------------------------------------ pieces of one solve
// Used by the uneven batch (ensemble.hip), which runs the inner iterations of
// several lattices together and these steps per lattice.
SolveFields solve_fields(lq_ctx* ctx, int inner) {
  Work* w = work(ctx, inner);
  work(ctx, LQ_F64);
  SolveFields f;
  f.x = w->x;
  f.bhat = w->bhat;
  f.r64 = w->r64;
  f.rn64 = w->rn64;
  f.to = w->to;
  f.p = w->p[inner];
  f.q = w->q[inner];
  f.t = w->t[inner];
  f.xl = w->xl[inner];
  f.r = w->r[inner];
  f.rt = w->rt[inner];
  return f;
}

double solve_begin(lq_ctx* ctx, void* dev_x, const void* dev_b, double* bhat_norm) {
  Work* w = work(ctx, LQ_F64);
  w->b = const_cast<void*>(dev_b);
  w->x = dev_x;
  double bn = 0.0;
  const double b2 = prepare_rhs(ctx, w, bn);
  *bhat_norm = bn;
  return b2;
}

bool solve_more(lq_ctx* ctx, int inner, double target, int maxiter, int check_every,
                bool use_graph, SolveTally& t) {
  Work* w = work(ctx, inner);
  SolveStats ss;
  bool fb = false;
  const double delta = inner == LQ_F64 ? 0.0 : 0.1;
  bool conv = run_cg(ctx, w, inner, target, delta, std::max(1, maxiter), check_every, use_graph,
                     0, ss, fb, nullptr);
  t.iterations += ss.iterations;
  t.reliable += ss.reliable;
  t.dslash += ss.dslash + 4 * ss.iterations;
  if (fb) {
    t.fallback = 1;
    work(ctx, LQ_F64);
    SolveStats f;
    conv = run_cg(ctx, w, LQ_F64, target, 0.0, std::max(1, maxiter - ss.iterations), check_every,
                  use_graph, 0, f, fb, nullptr);
    t.iterations += f.iterations;
    t.reliable += f.reliable;
    t.dslash += f.dslash + 4 * f.iterations;
  }
  return conv;
}

double solve_end(lq_ctx* ctx, double* schur2, SolveTally& t) {
  Work* w = ctx->work;
  SolveStats ss;
  const double res2 = reconstruct_and_residual(ctx, w, ss);
  *schur2 = schur_residual(ctx, w, ss);
  t.dslash += ss.dslash;
  return res2;
}

void iteration_bytes(int inner, double out[LQ_NK]) {
  iteration_site_bytes(inner, vec_prec(inner), out);
}

}  // namespace lq
