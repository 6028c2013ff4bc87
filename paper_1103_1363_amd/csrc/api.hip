// C ABI entry points (include/lq.h): argument checks, error capture, context
// lifetime.  No C++ exception crosses this boundary.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "lq_internal.h"
#include "reduce.h"

namespace {

thread_local std::string g_create_error;

template <class F>
lq_status guarded(lq_ctx* ctx, F&& f) {
  if (!ctx) return LQ_EINVAL;
  hipStream_t saved = ctx->cur;
  try {
    f();
    ctx->cur = saved;
    return LQ_OK;
  } catch (const lq::Error& e) {
    ctx->cur = saved;
    ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->cur = saved;
    ctx->err = "host allocation failed";
    return LQ_ENOMEM;
  } catch (const std::exception& e) {
    ctx->cur = saved;
    ctx->err = e.what();
    return LQ_EINVAL;
  }
}

void check_parity(int parity, bool allow_full) {
  LQ_CHECK(parity == LQ_EVEN || parity == LQ_ODD || (allow_full && parity == LQ_FULL), LQ_EINVAL,
           "bad parity");
}
void check_prec(int prec) {
  LQ_CHECK(prec == LQ_F64 || prec == LQ_F32 || prec == LQ_F16, LQ_EINVAL, "bad precision");
}
// LQ_F16X (multi-RHS interleaved) fields: one parity, at most 16 RHS
bool multi_rhs(int prec, int parity, int nrhs) {
  if (prec != LQ_F16X) return false;
  LQ_CHECK(parity == LQ_EVEN || parity == LQ_ODD, LQ_EINVAL,
           "multi-RHS fields hold one parity");
  LQ_CHECK(nrhs >= 1 && nrhs <= 16, LQ_EINVAL, "multi-RHS fields hold 1..16 right-hand sides");
  return true;
}

}  // namespace

namespace lq {

// Largest number of sites of one parity per tile; LQ_TILE_SITES overrides
// the default (tuning experiments).
int64_t tile_target() {
  const char* e = std::getenv("LQ_TILE_SITES");
  if (e) {
    const long long v = std::atoll(e);
    if (v >= 64) return v;
  }
  // measured on MI355X at 32^3x64: 65536 beats 4096, 16384 and untiled
  return 65536;
}

// Largest number of sites of one parity per tile of the multi-RHS fields;
// LQ_MR_TILE_SITES overrides the default (tuning experiments).
int64_t mr_tile_target() {
  const char* e = std::getenv("LQ_MR_TILE_SITES");
  if (e) {
    const long long v = std::atoll(e);
    if (v >= 64) return v;
  }
  return 2048;
}

size_t field_bytes(const lq_ctx* ctx, int parity, int prec, int nrhs) {
  size_t one = parity_field_bytes(ctx->geo.nblk, prec);
  return one * (parity == LQ_FULL ? 2 : 1) * (size_t)(nrhs > 0 ? nrhs : 1);
}

void* staging(lq_ctx* ctx, size_t bytes) {
  if (ctx->staging_bytes < bytes) {
    if (ctx->staging) {
      LQ_HIP(hipStreamSynchronize(ctx->cur));
      (void)hipFree(ctx->staging);
      ctx->staging = nullptr;
      ctx->staging_bytes = 0;
    }
    LQ_HIP(hipMalloc(&ctx->staging, bytes));
    ctx->staging_bytes = bytes;
  }
  return ctx->staging;
}

void ensure_red(lq_ctx* ctx) {
  if (!ctx->red) {
    LQ_HIP(hipMalloc(&ctx->red, RED_BYTES));
    LQ_HIP(hipMemsetAsync(ctx->red, 0, RED_BYTES, ctx->cur));
  }
}

}  // namespace lq

// the public net handle: the library net and the context it belongs to
struct lq_ensemble {
  lq::Ensemble* impl;
  std::string err;
};

struct lq_net {
  lq_ctx* ctx;
  lq::Net* impl;
};

extern "C" {

lq_status lq_create(const int dims[4], int t_antiperiodic, void* hip_stream, lq_ctx** out) {
  if (!out || !dims) {
    g_create_error = "null argument";
    return LQ_EINVAL;
  }
  *out = nullptr;
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || (dims[k] & 1)) {
      g_create_error = "every lattice extent must be even and >= 2";
      return LQ_EINVAL;
    }
  const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
  if (V / 2 > (int64_t)lq::RED_MAX_BLOCKS * 256) {
    g_create_error = "lattice too large for the reduction scratch";
    return LQ_EINVAL;
  }
  int device = 0;
  const hipError_t de = hipGetDevice(&device);
  if (de != hipSuccess) {
    g_create_error = std::string("hipGetDevice failed: ") + hipGetErrorString(de);
    return LQ_EHIP;
  }
  try {
    lq::noalloc_init(device);  // address of the no-allocation scratch array on this device
  } catch (const lq::Error& e) {
    g_create_error = e.what();
    return e.code;
  }
  lq_ctx* ctx = new (std::nothrow) lq_ctx();
  if (!ctx) return LQ_ENOMEM;
  ctx->device = device;
  for (int k = 0; k < 4; ++k) {
    ctx->dims[k] = dims[k];
    ctx->geo.L[k] = dims[k];
  }
  lq::choose_tiles(ctx->geo.L, lq::tile_target(), ctx->geo.T);
  lq::geo_finish(ctx->geo);
  ctx->geo.apt = t_antiperiodic ? 1 : 0;
  ctx->mr_geo = ctx->geo;
  lq::choose_tiles(ctx->geo.L, lq::mr_tile_target(), ctx->mr_geo.T);
  lq::geo_finish(ctx->mr_geo);
  ctx->V = V;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->cur = ctx->stream;
  const hipError_t se = hipStreamCreateWithFlags(&ctx->sstream, hipStreamNonBlocking);
  if (se != hipSuccess) {
    g_create_error = std::string("hipStreamCreateWithFlags failed: ") + hipGetErrorName(se) +
                     " (" + hipGetErrorString(se) + ")";
    delete ctx;
    return LQ_EHIP;
  }
  *out = ctx;
  return LQ_OK;
}

void lq_destroy(lq_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  (void)hipStreamSynchronize(ctx->sstream);
  lq::free_work(ctx);
  lq::free_mrhs_work(ctx);
  lq::free_mrhs_tables(ctx);
  lq::free_clover(ctx);
  lq::sap_destroy(ctx->sap);
  lq::free_krylov(ctx);
  lq::free_block_work(ctx);
  for (int p = 0; p < 3; ++p)
    if (ctx->gauge[p]) (void)hipFree(ctx->gauge[p]);
  if (ctx->staging) (void)hipFree(ctx->staging);
  if (ctx->red) (void)hipFree(ctx->red);
  (void)hipStreamDestroy(ctx->sstream);
  delete ctx;
}

const char* lq_last_error(const lq_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

size_t lq_field_bytes(const lq_ctx* ctx, int parity, int prec, int nrhs) {
  if (!ctx || (parity != LQ_EVEN && parity != LQ_ODD && parity != LQ_FULL) || prec < 0 ||
      prec > 3 || nrhs < 1)
    return 0;
  if (prec == LQ_F16X) return (parity == LQ_FULL || nrhs > 16) ? 0 : lq::mr_field_bytes(ctx, nrhs);
  return lq::field_bytes(ctx, parity, prec, nrhs);
}

int64_t lq_volume(const lq_ctx* ctx) { return ctx ? ctx->V : 0; }

lq_status lq_upload_gauge(lq_ctx* ctx, const double* host_U) {
  return guarded(ctx, [&] {
    LQ_CHECK(host_U, LQ_EINVAL, "null gauge pointer");
    lq::upload_gauge(ctx, host_U);
  });
}

lq_status lq_set_clover(lq_ctx* ctx, double kappa, double csw) {
  return guarded(ctx, [&] {
    LQ_CHECK(kappa > 0.0 && kappa < 0.25, LQ_EINVAL, "kappa must lie in (0, 0.25)");
    LQ_CHECK(csw >= 0.0, LQ_EINVAL, "csw must be >= 0");
    lq::build_clover(ctx, kappa, csw);
  });
}

lq_status lq_spinor_to_device(lq_ctx* ctx, void* dev, const double* host, int parity, int prec,
                              int nrhs) {
  return guarded(ctx, [&] {
    LQ_CHECK(dev && host && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    check_parity(parity, true);
    if (multi_rhs(prec, parity, nrhs)) {
      const size_t hb = (size_t)ctx->geo.vh * 12 * 16;
      double2* st = reinterpret_cast<double2*>(lq::staging(ctx, hb));
      for (int r = 0; r < nrhs; ++r) {
        LQ_HIP(hipMemcpyAsync(st, host + (size_t)r * ctx->geo.vh * 24, hb, hipMemcpyHostToDevice,
                              ctx->cur));
        lq::mrhs_pack(ctx, dev, st, parity, LQ_F16, nrhs, r);
      }
      LQ_HIP(hipStreamSynchronize(ctx->cur));
      return;
    }
    check_prec(prec);
    const int full = parity == LQ_FULL;
    const int64_t nsites = full ? ctx->V : ctx->geo.vh;
    const size_t hb = (size_t)nsites * 12 * 16;
    const size_t fb = lq::field_bytes(ctx, parity, prec, 1);
    double2* st = reinterpret_cast<double2*>(lq::staging(ctx, hb));
    for (int r = 0; r < nrhs; ++r) {
      LQ_HIP(hipMemcpyAsync(st, host + (size_t)r * nsites * 24, hb, hipMemcpyHostToDevice,
                            ctx->cur));
      lq::pack_spinor(ctx, reinterpret_cast<char*>(dev) + r * fb, st, prec, parity);
    }
    LQ_HIP(hipStreamSynchronize(ctx->cur));
  });
}

lq_status lq_spinor_to_host(lq_ctx* ctx, double* host, const void* dev, int parity, int prec,
                            int nrhs) {
  return guarded(ctx, [&] {
    LQ_CHECK(dev && host && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    check_parity(parity, true);
    if (multi_rhs(prec, parity, nrhs)) {
      const size_t hb = (size_t)ctx->geo.vh * 12 * 16;
      double2* st = reinterpret_cast<double2*>(lq::staging(ctx, hb));
      for (int r = 0; r < nrhs; ++r) {
        lq::mrhs_unpack(ctx, st, dev, parity, LQ_F16, nrhs, r);
        LQ_HIP(hipMemcpyAsync(host + (size_t)r * ctx->geo.vh * 24, st, hb, hipMemcpyDeviceToHost,
                              ctx->cur));
        LQ_HIP(hipStreamSynchronize(ctx->cur));
      }
      return;
    }
    check_prec(prec);
    const int full = parity == LQ_FULL;
    const int64_t nsites = full ? ctx->V : ctx->geo.vh;
    const size_t hb = (size_t)nsites * 12 * 16;
    const size_t fb = lq::field_bytes(ctx, parity, prec, 1);
    double2* st = reinterpret_cast<double2*>(lq::staging(ctx, hb));
    for (int r = 0; r < nrhs; ++r) {
      lq::unpack_spinor(ctx, st, reinterpret_cast<const char*>(dev) + r * fb, prec, parity);
      LQ_HIP(hipMemcpyAsync(host + (size_t)r * nsites * 24, st, hb, hipMemcpyDeviceToHost,
                            ctx->cur));
      LQ_HIP(hipStreamSynchronize(ctx->cur));
    }
  });
}

lq_status lq_dslash(lq_ctx* ctx, void* dev_out, const void* dev_in, int out_parity, int dagger,
                    int prec, int nrhs) {
  return guarded(ctx, [&] {
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    LQ_CHECK(dev_out && dev_in && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    LQ_CHECK(dev_out != dev_in, LQ_EINVAL, "dslash cannot run in place");
    check_parity(out_parity, false);
    if (multi_rhs(prec, out_parity, nrhs)) {
      LQ_CHECK(ctx->gauge[LQ_F16], LQ_ESTATE, "no FP16 gauge field");
      lq::mrhs_dslash(ctx, dev_out, dev_in, out_parity, dagger, nrhs);
      return;
    }
    check_prec(prec);
    const size_t fb = lq::field_bytes(ctx, LQ_EVEN, prec, 1);
    for (int r = 0; r < nrhs; ++r)
      lq::dslash(ctx, reinterpret_cast<char*>(dev_out) + r * fb,
                 reinterpret_cast<const char*>(dev_in) + r * fb, out_parity, dagger, prec);
  });
}

lq_status lq_clover_apply(lq_ctx* ctx, void* dev_out, const void* dev_in, int parity, int inverse,
                          int prec, int nrhs) {
  return guarded(ctx, [&] {
    LQ_CHECK(ctx->clov.valid, LQ_ESTATE, "no clover term (call lq_set_clover)");
    LQ_CHECK(dev_out && dev_in && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    check_parity(parity, false);
    check_prec(prec);
    const size_t fb = lq::field_bytes(ctx, LQ_EVEN, prec, 1);
    for (int r = 0; r < nrhs; ++r)
      lq::clover_apply(ctx, reinterpret_cast<char*>(dev_out) + r * fb,
                       reinterpret_cast<const char*>(dev_in) + r * fb, parity, inverse, prec);
  });
}

lq_status lq_schur(lq_ctx* ctx, void* dev_out, const void* dev_in, void* dev_tmp, int dagger,
                   int prec, int nrhs) {
  return guarded(ctx, [&] {
    LQ_CHECK(ctx->clov.valid, LQ_ESTATE, "no clover term (call lq_set_clover)");
    LQ_CHECK(dev_out && dev_in && dev_tmp && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    LQ_CHECK(dev_out != dev_in && dev_tmp != dev_in && dev_tmp != dev_out, LQ_EINVAL,
             "schur needs three distinct buffers");
    if (multi_rhs(prec, LQ_EVEN, nrhs)) {
      lq::mrhs_schur(ctx, dev_out, dev_in, dev_tmp, dagger, nrhs);
      return;
    }
    check_prec(prec);
    const size_t fb = lq::field_bytes(ctx, LQ_EVEN, prec, 1);
    for (int r = 0; r < nrhs; ++r)
      lq::schur(ctx, reinterpret_cast<char*>(dev_out) + r * fb,
                reinterpret_cast<const char*>(dev_in) + r * fb,
                reinterpret_cast<char*>(dev_tmp) + r * fb, dagger, prec);
  });
}

lq_status lq_schur_noalloc(lq_ctx* ctx, void* dev_out, const void* dev_in, int dagger,
                           int prec, int nrhs) {
  return guarded(ctx, [&] {
    LQ_CHECK(dev_out && dev_in && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    LQ_CHECK(dev_out != dev_in, LQ_EINVAL, "schur needs distinct input and output buffers");
    lq::schur_noalloc(ctx, dev_out, dev_in, dagger, prec, nrhs);
  });
}

lq_status lq_norm2(lq_ctx* ctx, double* out, const void* dev_a, int parity, int prec) {
  return guarded(ctx, [&] {
    LQ_CHECK(out && dev_a, LQ_EINVAL, "null pointer");
    check_parity(parity, false);
    check_prec(prec);
    lq::norm2(ctx, out, dev_a, prec);
  });
}

lq_status lq_dot(lq_ctx* ctx, double* out, const void* dev_a, const void* dev_b, int parity,
                 int prec) {
  return guarded(ctx, [&] {
    LQ_CHECK(out && dev_a && dev_b, LQ_EINVAL, "null pointer");
    check_parity(parity, false);
    check_prec(prec);
    lq::dot(ctx, out, dev_a, dev_b, prec);
  });
}

lq_status lq_solve(lq_ctx* ctx, double* host_x, const double* host_b, int nrhs, double kappa,
                   double csw, double tol, const lq_solver_params* params,
                   lq_solve_report* report) {
  return guarded(ctx, [&] {
    LQ_CHECK(host_x && host_b && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    LQ_CHECK(kappa > 0.0 && kappa < 0.25 && csw >= 0.0, LQ_EINVAL, "bad kappa or csw");
    LQ_CHECK(tol > 0.0 && tol < 1.0, LQ_EINVAL, "tol must lie in (0, 1)");
    lq::solve(ctx, host_x, host_b, nullptr, nullptr, nrhs, kappa, csw, tol, params, report);
  });
}

lq_status lq_solve_device(lq_ctx* ctx, void* dev_x, const void* dev_b, int nrhs, double kappa,
                          double csw, double tol, const lq_solver_params* params,
                          lq_solve_report* report) {
  return guarded(ctx, [&] {
    LQ_CHECK(dev_x && dev_b && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    LQ_CHECK(dev_x != dev_b, LQ_EINVAL, "x and b must be distinct buffers");
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    LQ_CHECK(kappa > 0.0 && kappa < 0.25 && csw >= 0.0, LQ_EINVAL, "bad kappa or csw");
    LQ_CHECK(tol > 0.0 && tol < 1.0, LQ_EINVAL, "tol must lie in (0, 1)");
    lq::solve(ctx, nullptr, nullptr, dev_x, dev_b, nrhs, kappa, csw, tol, params, report);
  });
}

// ------------------------------------------------------------ SAP and FGCR
lq_status lq_sap_apply(lq_ctx* ctx, void* dev_out, const void* dev_in,
                       const lq_sap_params* params) {
  return guarded(ctx, [&] {
    LQ_CHECK(dev_out && dev_in && params, LQ_EINVAL, "null pointer");
    LQ_CHECK(dev_out != dev_in, LQ_EINVAL, "in and out must be distinct buffers");
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    lq::sap_apply(ctx, dev_out, dev_in, *params);
  });
}

lq_status lq_solve_sap(lq_ctx* ctx, void* dev_x, const void* dev_b, double kappa, double csw,
                       double tol, const lq_sap_params* params, lq_solve_report* report) {
  return guarded(ctx, [&] {
    LQ_CHECK(dev_x && dev_b && params, LQ_EINVAL, "null pointer");
    LQ_CHECK(dev_x != dev_b, LQ_EINVAL, "x and b must be distinct buffers");
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    LQ_CHECK(kappa > 0.0 && kappa < 0.25 && csw >= 0.0, LQ_EINVAL, "bad kappa or csw");
    LQ_CHECK(tol > 0.0 && tol < 1.0, LQ_EINVAL, "tol must lie in (0, 1)");
    // after the caller's work, on the library stream
    if (ctx->stream) LQ_HIP(hipStreamSynchronize(ctx->stream));
    else LQ_HIP(hipDeviceSynchronize());
    ctx->cur = ctx->sstream;
    if (!ctx->clov.valid || ctx->clov.kappa != kappa || ctx->clov.csw != csw)
      lq::build_clover(ctx, kappa, csw);
    const bool dr = params->deflate > 0;
    const bool ok = dr ? lq::solve_sap_dr(ctx, dev_x, dev_b, tol, *params, report)
                       : lq::solve_sap(ctx, dev_x, dev_b, tol, *params, report);
    LQ_CHECK(ok, LQ_ENOCONV,
             dr ? "SAP-FGMRES-DR did not reach the tolerance" : "SAP-FGCR did not reach the tolerance");
  });
}

// ------------------------------------------------------------ learned preconditioner
lq_status lq_net_create(lq_ctx* ctx, int nlayers, lq_net** out) {
  return guarded(ctx, [&] {
    LQ_CHECK(out, LQ_EINVAL, "null pointer");
    lq::Net* n = lq::net_create(ctx, nlayers);
    *out = new lq_net{ctx, n};
  });
}

void lq_net_destroy(lq_net* net) {
  if (!net) return;
  (void)hipStreamSynchronize(net->ctx->cur);
  lq::net_destroy(net->impl);
  delete net;
}

lq_status lq_net_set_weights(lq_net* net, const double* host_w) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(host_w, LQ_EINVAL, "null pointer");
    lq::net_set_weights(net->impl, host_w);
  });
}

lq_status lq_net_init_neumann(lq_net* net, double kappa) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(std::isfinite(kappa), LQ_EINVAL, "bad kappa");
    lq::net_init_neumann(net->impl, kappa);
  });
}

lq_status lq_net_get_weights(lq_net* net, double* host_w) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(host_w, LQ_EINVAL, "null pointer");
    lq::net_get_weights(net->impl, host_w);
  });
}

lq_status lq_net_apply(lq_net* net, void* dev_out, const void* dev_in, int mode) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(dev_out && dev_in && dev_out != dev_in, LQ_EINVAL,
             "null or identical device pointers");
    LQ_CHECK(mode >= 0 && mode <= 3, LQ_EINVAL, "bad mode");
    if (mode & LQ_NET_FP16)
      lq::net_apply_even_fast(net->impl, dev_out, dev_in, (mode & LQ_NET_ADJOINT) != 0);
    else
      lq::net_apply_even(net->impl, dev_out, dev_in, (mode & LQ_NET_ADJOINT) != 0);
    LQ_HIP(hipStreamSynchronize(net->ctx->cur));
  });
}

lq_status lq_net_loss_grad(lq_net* net, const void* dev_b, const void* dev_x, int npairs,
                           double* loss, double* host_grad) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(dev_b && dev_x && loss && npairs >= 1, LQ_EINVAL, "null pointer or npairs < 1");
    *loss = lq::net_loss_grad(net->impl, dev_b, dev_x, npairs);
    if (host_grad) lq::net_get_grad(net->impl, host_grad);
  });
}

lq_status lq_net_adam_step(lq_net* net, double lr, double beta1, double beta2, double eps) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(lr > 0.0 && beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0,
             LQ_EINVAL, "bad Adam parameters");
    lq::net_adam(net->impl, lr, beta1, beta2, eps);
    LQ_HIP(hipStreamSynchronize(net->ctx->cur));
  });
}

lq_status lq_net_train(lq_net* net, const void* dev_b, const void* dev_x, int npairs, int epochs,
                       int batch, double lr, unsigned seed, double* loss_history) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] {
    LQ_CHECK(dev_b && dev_x, LQ_EINVAL, "null pointer");
    LQ_CHECK(lr > 0.0, LQ_EINVAL, "bad learning rate");
    lq::net_train(net->impl, dev_b, dev_x, npairs, epochs, batch, lr, seed, loss_history);
    LQ_HIP(hipStreamSynchronize(net->ctx->cur));
  });
}

lq_status lq_net_save(lq_net* net, const char* path) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] { lq::net_save(net->impl, path); });
}

lq_status lq_net_load(lq_net* net, const char* path) {
  if (!net) return LQ_EINVAL;
  return guarded(net->ctx, [&] { lq::net_load(net->impl, path); });
}

lq_status lq_solve_net(lq_ctx* ctx, lq_net* net, double* host_x, const double* host_b, int nrhs,
                       double kappa, double csw, double tol, const lq_solver_params* params,
                       lq_solve_report* report) {
  return guarded(ctx, [&] {
    LQ_CHECK(net && host_x && host_b && nrhs >= 1, LQ_EINVAL, "null pointer or nrhs < 1");
    LQ_CHECK(net->ctx == ctx, LQ_EINVAL, "the net belongs to another context");
    LQ_CHECK(params && (params->solver == LQ_FGMRES_NET || params->solver == LQ_FCG_NET),
             LQ_EINVAL, "params->solver must be LQ_FGMRES_NET or LQ_FCG_NET");
    LQ_CHECK(ctx->have_gauge, LQ_ESTATE, "no gauge field uploaded");
    LQ_CHECK(kappa > 0.0 && kappa < 0.25 && csw >= 0.0, LQ_EINVAL, "bad kappa or csw");
    LQ_CHECK(tol > 0.0 && tol < 1.0, LQ_EINVAL, "tol must lie in (0, 1)");
    lq::solve(ctx, host_x, host_b, nullptr, nullptr, nrhs, kappa, csw, tol, params, report,
              net->impl);
  });
}

}  // extern "C"

// ------------------------------------------------------------ uneven batch
namespace {
thread_local std::string g_ens_create_error;

template <class F>
lq_status guarded_e(lq_ensemble* e, F&& f) {
  if (!e) return LQ_EINVAL;
  try {
    f();
    return LQ_OK;
  } catch (const lq::Error& x) {
    e->err = x.what();
    return x.code;
  } catch (const std::bad_alloc&) {
    e->err = "host allocation failed";
    return LQ_ENOMEM;
  } catch (const std::exception& x) {
    e->err = x.what();
    return LQ_EINVAL;
  }
}
}  // namespace

extern "C" {

lq_status lq_ensemble_create(lq_ctx* const* members, int n, lq_ensemble** out) {
  if (!out) {
    g_ens_create_error = "null pointer";
    return LQ_EINVAL;
  }
  *out = nullptr;
  try {
    lq::Ensemble* impl = lq::ensemble_create(members, n);
    *out = new lq_ensemble{impl, std::string()};
    return LQ_OK;
  } catch (const lq::Error& x) {
    g_ens_create_error = x.what();
    return x.code;
  } catch (const std::exception& x) {
    g_ens_create_error = x.what();
    return LQ_ENOMEM;
  }
}

void lq_ensemble_destroy(lq_ensemble* e) {
  if (!e) return;
  lq::ensemble_destroy(e->impl);
  delete e;
}

const char* lq_ensemble_last_error(const lq_ensemble* e) {
  return e ? e->err.c_str() : g_ens_create_error.c_str();
}

lq_status lq_ensemble_tune(lq_ensemble* e, int inner_prec, const char* cache_path,
                           lq_ensemble_report* rep) {
  return guarded_e(e, [&] { lq::ensemble_tune(e->impl, inner_prec, cache_path, rep); });
}

lq_status lq_ensemble_solve(lq_ensemble* e, void* const* dev_x, const void* const* dev_b,
                            const double* kappa, const double* csw, double tol,
                            const lq_solver_params* params, lq_solve_report* reports,
                            lq_ensemble_report* rep) {
  return guarded_e(e, [&] {
    LQ_CHECK(dev_x && dev_b && kappa && csw, LQ_EINVAL, "null pointer");
    LQ_CHECK(tol > 0.0 && tol < 1.0, LQ_EINVAL, "tol must lie in (0, 1)");
    lq::ensemble_solve(e->impl, dev_x, dev_b, kappa, csw, tol, params, reports, rep);
  });
}

}  // extern "C"
