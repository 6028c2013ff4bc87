// The Schur operator for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): lq_schur_noalloc keeps the odd-parity intermediate
// t = A_oo^-1 H_oe in, which lq_schur takes as a caller buffer, in a
// file-scope device array instead.
//
// The array is a host-side stand-in in host code: its device address is
// taken once per device with hipGetSymbolAddress (at lq_create, with the
// context's device current) and only that address is handed to kernels.
// Every GPU holds its own copy until the process ends, and every call on a
// GPU shares it: calls that overlap in time on one GPU race.  Nothing in it
// must start at zero (the first kernel writes every odd site the second one
// reads), so it is never cleared.
#include <mutex>

#include "lq_internal.h"

namespace lq {

namespace {

__device__ __align__(256) unsigned char scratch[LQ_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

void noalloc_init(int device) {
  LQ_CHECK(device >= 0 && device < kMaxDevices, LQ_EINVAL,
           "device ordinal beyond the scratch address table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  LQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  LQ_CHECK(p != nullptr, LQ_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[device] = p;
}

void schur_noalloc(lq_ctx* ctx, void* out, const void* in, int dagger, int prec, int nrhs) {
  LQ_CHECK(prec == LQ_F64 || prec == LQ_F32 || prec == LQ_F16, LQ_EINVAL,
           "lq_schur_noalloc: precision must be LQ_F64, LQ_F32 or LQ_F16 (the multi-RHS "
           "operator needs tables the library allocates)");
  const size_t fb = parity_field_bytes(ctx->geo.nblk, prec);
  LQ_CHECK(fb <= (size_t)LQ_SCRATCH_BYTES, LQ_EINVAL,
           "lq_schur_noalloc: one odd field of this lattice and precision needs " +
               std::to_string(fb) + " bytes, above the " + std::to_string(LQ_SCRATCH_BYTES) +
               "-byte scratch array");
  LQ_CHECK(ctx->clov.valid, LQ_ESTATE, "no clover term (call lq_set_clover)");
  void* tmp = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    tmp = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
  }
  LQ_CHECK(tmp != nullptr, LQ_ESTATE, "scratch array address not resolved for this device");
  // the right-hand sides run one after another on one stream and share t
  for (int r = 0; r < nrhs; ++r)
    schur(ctx, reinterpret_cast<char*>(out) + r * fb, reinterpret_cast<const char*>(in) + r * fb,
          tmp, dagger, prec);
}

}  // namespace lq
