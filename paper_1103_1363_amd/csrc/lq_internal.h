// Internal declarations of the lq library: context, device layouts, the
// complex arithmetic and precision traits shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lq.h"

#define LQ_HD __host__ __device__
#include "site_index.h"

namespace lq {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  lq_status code;
  Error(lq_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define LQ_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::lq::Error(LQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LQ_CHECK(cond, code, msg)                     \
  do {                                                \
    if (!(cond)) throw ::lq::Error((code), (msg));    \
  } while (0)

// ---------------------------------------------------------------- layout
// Sites of one parity are numbered by their checkerboard index s = i / 2
// (i the full-lattice index).  Device fields group sites into blocks of 64;
// inside a block each complex component occupies 64 consecutive slots, so
// the 64 lanes of a wavefront read one component of 64 consecutive sites
// with a single coalesced load.
constexpr int SB = 64;  // sites per block

__host__ __device__ inline int64_t spin_idx(int64_t s, int c) {  // c in [0, 12)
  return ((s >> 6) * 12 + c) * SB + (s & 63);
}
__host__ __device__ inline int64_t clov_idx(int64_t s, int c) {  // c in [0, 36)
  return ((s >> 6) * 36 + c) * SB + (s & 63);
}
// compressed links: parity p, direction mu, site s, complex entry c in [0, 6)
// (row 0 then row 1)
__host__ __device__ inline int64_t link_idx(int64_t nblk, int p, int mu, int64_t s, int c) {
  return ((((int64_t)p * 4 + mu) * nblk + (s >> 6)) * 6 + c) * SB + (s & 63);
}


// ---------------------------------------------------------------- complex
template <class R>
struct C {
  R re, im;
};
template <class R>
__device__ __forceinline__ C<R> cmk(R a, R b) { return C<R>{a, b}; }
template <class R>
__device__ __forceinline__ C<R> operator+(C<R> a, C<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ C<R> operator-(C<R> a, C<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ C<R> operator-(C<R> a) { return {-a.re, -a.im}; }
template <class R>
__device__ __forceinline__ C<R> operator*(C<R> a, C<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__device__ __forceinline__ C<R> operator*(R s, C<R> a) { return {s * a.re, s * a.im}; }
template <class R>
__device__ __forceinline__ C<R> conj(C<R> a) { return {a.re, -a.im}; }
template <class R>
__device__ __forceinline__ C<R> times_i(C<R> a) { return {-a.im, a.re}; }
// conj(a) * b
template <class R>
__device__ __forceinline__ C<R> cmul_conj(C<R> a, C<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class R>
__device__ __forceinline__ R norm2(C<R> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------- precision traits
// Register budget of the hopping kernels: at least this many waves per SIMD
// (512 / waves VGPRs per lane).  The compiler otherwise hoists all eight
// neighbour loads and trades occupancy for instruction-level parallelism,
// which loses on these bandwidth-bound kernels.
#ifndef LQ_WAVES_F64
#define LQ_WAVES_F64 2
#endif
#ifndef LQ_WAVES_F32
#define LQ_WAVES_F32 4
#endif
#ifndef LQ_WAVES_F16
#define LQ_WAVES_F16 3
#endif
#define LQ_HOP_KERNEL(P) \
  __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P::waves)))
// Storage type S, arithmetic type R.  FP16 fields hold fp16(value / scale)
// with one FP32 scale per site stored after the component array.
struct P64 {
  using R = double;
  using S = double2;
  static constexpr bool has_norm = false;
  static constexpr int id = LQ_F64;
  static constexpr int waves = LQ_WAVES_F64;  // minimum waves per SIMD of hopping kernels
};
struct P32 {
  using R = float;
  using S = float2;
  static constexpr bool has_norm = false;
  static constexpr int id = LQ_F32;
  static constexpr int waves = LQ_WAVES_F32;
};
struct P16 {
  using R = float;
  using S = __half2;
  static constexpr bool has_norm = true;
  static constexpr int id = LQ_F16;
  static constexpr int waves = LQ_WAVES_F16;
};

template <class P>
__device__ __forceinline__ C<typename P::R> ld(const typename P::S* p, int64_t i);
template <>
__device__ __forceinline__ C<double> ld<P64>(const double2* p, int64_t i) {
  double2 v = p[i];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ld<P32>(const float2* p, int64_t i) {
  float2 v = p[i];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ld<P16>(const __half2* p, int64_t i) {
  float2 v = __half22float2(p[i]);
  return {v.x, v.y};
}
// Streaming loads for data read exactly once per sweep (links, clover
// tables): the non-temporal hint lets L2 keep the spinors, which are read
// by eight neighbours, instead of the streamed tables.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u1;
template <class P>
__device__ __forceinline__ C<typename P::R> ldnt(const typename P::S* p, int64_t i);
template <>
__device__ __forceinline__ C<double> ldnt<P64>(const double2* p, int64_t i) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p) + i);
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ldnt<P32>(const float2* p, int64_t i) {
  const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p) + i);
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ C<float> ldnt<P16>(const __half2* p, int64_t i) {
  const nt_u1 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u1*>(p) + i);
  __half2 h;
  __builtin_memcpy(&h, &v, 4);
  const float2 f = __half22float2(h);
  return {f.x, f.y};
}

template <class P>
__device__ __forceinline__ void st(typename P::S* p, int64_t i, C<typename P::R> v);
template <>
__device__ __forceinline__ void st<P64>(double2* p, int64_t i, C<double> v) {
  p[i] = make_double2(v.re, v.im);
}
template <>
__device__ __forceinline__ void st<P32>(float2* p, int64_t i, C<float> v) {
  p[i] = make_float2(v.re, v.im);
}
template <>
__device__ __forceinline__ void st<P16>(__half2* p, int64_t i, C<float> v) {
  p[i] = __floats2half2_rn(v.re, v.im);
}

// A device spinor field of one parity (and one right-hand side).
template <class P>
struct Field {
  typename P::S* d;
  float* norm;  // FP16 only: per-site scale
};

// bytes of one parity field of vh sites for precision prec
inline size_t parity_field_bytes(int64_t nblk, int prec) {
  int64_t n = nblk * SB;
  switch (prec) {
    case LQ_F64: return (size_t)n * 12 * 16;
    case LQ_F32: return (size_t)n * 12 * 8;
    default: return (size_t)n * 12 * 4 + (size_t)n * 4;
  }
}

template <class P>
__host__ __device__ inline Field<P> field_at(void* base, int64_t nblk) {
  Field<P> f;
  f.d = reinterpret_cast<typename P::S*>(base);
  f.norm = P::has_norm ? reinterpret_cast<float*>(reinterpret_cast<char*>(base) +
                                                  (size_t)nblk * SB * 12 * 4)
                       : nullptr;
  return f;
}

// Load the 12 components of site s (spin-major, colour-minor).
template <class P>
__device__ __forceinline__ void load_spinor(const Field<P>& f, int64_t s,
                                            C<typename P::R> v[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = ld<P>(f.d, spin_idx(s, c));
  if constexpr (P::has_norm) {
    float n = f.norm[s];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = n * v[c];
  }
}
template <class P>
__device__ __forceinline__ void store_spinor(const Field<P>& f, int64_t s,
                                             C<typename P::R> v[12]) {
  if constexpr (P::has_norm) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    f.norm[s] = m;
    float inv = m > 0.f ? 1.f / m : 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) st<P>(f.d, spin_idx(s, c), inv * v[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) st<P>(f.d, spin_idx(s, c), v[c]);
  }
}

// Load the 12 raw components of site s (FP16: without the scale) and the
// site scale (1 for FP64/FP32).
template <class P>
__device__ __forceinline__ typename P::R load_raw(const Field<P>& f, int64_t s,
                                                   C<typename P::R> v[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = ld<P>(f.d, spin_idx(s, c));
  if constexpr (P::has_norm)
    return f.norm[s];
  else
    return (typename P::R)1;
}

// ---------------------------------------------------------------- context
struct Clover {
  // FP64: A and A^{-1} for both parities; lower precisions: A_ee and A_oo^{-1}
  void* a64[2] = {nullptr, nullptr};
  void* ainv64[2] = {nullptr, nullptr};
  void* a_ee[3] = {nullptr, nullptr, nullptr};
  void* ainv_oo[3] = {nullptr, nullptr, nullptr};
  double kappa = 0, csw = 0;
  bool valid = false;
};

struct Work;    // solver work space (solver.hip)
struct MRWork;  // batched multi-RHS solver work space (mrhs.hip)
struct Net;     // learned preconditioner (net.hip)
struct Ensemble;  // uneven batch of independent solves (ensemble.hip)

}  // namespace lq

struct lq_ctx {
  lq::Geo geo;
  int dims[4];
  int64_t V;
  hipStream_t stream = nullptr;   // caller's stream (public per-operation calls)
  hipStream_t sstream = nullptr;  // library-owned stream used by the solvers
  hipStream_t cur = nullptr;      // stream the kernel wrappers launch on
  void* gauge[3] = {nullptr, nullptr, nullptr};  // compressed links per precision
  bool have_gauge = false;
  lq::Clover clov;
  void* staging = nullptr;  // FP64 host-layout staging buffer
  size_t staging_bytes = 0;
  void* red = nullptr;      // reduction scratch (partials + counter + result)
  lq::Work* work = nullptr;
  lq::MRWork* mrwork = nullptr;
  // FP16 site-major operator copies of the multi-RHS kernels (mrhs.hip)
  void* mr_links = nullptr;
  void* mr_nbr = nullptr;  // neighbour table (geometry only)
  void* mr_clov[2] = {nullptr, nullptr};  // A_ee (even sites), A_oo^-1 (odd sites)
  bool mr_links_ok = false, mr_clov_ok = false;
  std::string err;
  double bytes = 0.0;       // algorithmic bytes of every kernel launched so far
};

namespace lq {

// Reduction scratch layout (ctx->red): partial sums then a counter then results.
constexpr int RED_MAX_BLOCKS = 65536;
constexpr int RED_NVAL = 4;  // values reduced at once at most

size_t field_bytes(const lq_ctx* ctx, int parity, int prec, int nrhs);
void* staging(lq_ctx* ctx, size_t bytes);
void ensure_red(lq_ctx* ctx);

// layout.hip
void upload_gauge(lq_ctx* ctx, const double* host_U);
// parity: LQ_EVEN / LQ_ODD (host half field, dev one parity field) or
// LQ_FULL (host full field, dev = even half then odd half)
void pack_spinor(lq_ctx* ctx, void* dev, const double2* src_dev, int prec, int parity);
void unpack_spinor(lq_ctx* ctx, double2* dst_dev, const void* dev, int prec, int parity);

// dslash.hip
void dslash(lq_ctx* ctx, void* out, const void* in, int out_parity, int dagger, int prec);
void clover_apply(lq_ctx* ctx, void* out, const void* in, int parity, int inverse, int prec);
void schur(lq_ctx* ctx, void* out, const void* in, void* tmp, int dagger, int prec);

// clover.hip
void build_clover(lq_ctx* ctx, double kappa, double csw);
void free_clover(lq_ctx* ctx);

// blas.hip
void norm2(lq_ctx* ctx, double* out_host, const void* a, int prec);
void dot(lq_ctx* ctx, double* out_host, const void* a, const void* b, int prec);

// solver.hip
// host_x/host_b (host canonical arrays) or dev_x/dev_b (full-lattice FP64
// device fields); the unused pair is null.
void solve(lq_ctx* ctx, double* host_x, const double* host_b, void* dev_x, const void* dev_b,
           int nrhs, double kappa, double csw, double tol, const lq_solver_params* params,
           lq_solve_report* report, Net* net = nullptr);
void free_work(lq_ctx* ctx);
// Pieces of one solve, for the uneven batch (ensemble.hip): the work fields
// of inner precision `inner` (allocated on first use); right-hand side setup
// from a full-lattice FP64 device field (bhat, x = 0; returns |b|^2);
// a single-lattice continuation from the current x to the Schur target
// (mixed CG with the FP64 fallback); odd-site reconstruction with the full
// residual |b - M x|^2 and the Schur residual.
struct SolveFields {
  void *x, *bhat, *r64, *rn64, *to;  // FP64: x (full lattice, even half first), even, odd
  void *p, *q, *t, *xl, *r, *rt;     // inner iteration (t odd, the rest even)
};
struct SolveTally {
  int iterations = 0, reliable = 0, fallback = 0, dslash = 0;
};
SolveFields solve_fields(lq_ctx* ctx, int inner);
double solve_begin(lq_ctx* ctx, void* dev_x, const void* dev_b, double* bhat_norm);
bool solve_more(lq_ctx* ctx, int inner, double target, int maxiter, int check_every,
                bool use_graph, SolveTally& t);
double solve_end(lq_ctx* ctx, double* schur2, SolveTally& t);
void iteration_bytes(int inner, double out[LQ_NK]);  // per site, per kernel of one iteration

// mrhs.hip: multi-RHS interleaved FP16 fields (lq_prec LQ_F16X) and the
// matrix-core hopping term; batched CG helpers
size_t mr_field_bytes(const lq_ctx* ctx, int nrhs);
void mrhs_pack(lq_ctx* ctx, void* dev, const double2* src_dev, int parity, int prec, int nrhs,
               int r);
void mrhs_unpack(lq_ctx* ctx, double2* dst_dev, const void* dev, int parity, int prec, int nrhs,
                 int r);
void mrhs_dslash(lq_ctx* ctx, void* out, const void* in, int out_parity, int dagger, int nrhs);
void mrhs_schur(lq_ctx* ctx, void* out, const void* in, void* tmp, int dagger, int nrhs);
MRWork* mrhs_work(lq_ctx* ctx, int nrhs);
void free_mrhs_work(lq_ctx* ctx);
void mrhs_tables(lq_ctx* ctx, bool clover);  // build the FP16 operator copies if stale
void free_mrhs_tables(lq_ctx* ctx);

// net.hip: learned gauge-covariant preconditioner (FP32 even fields)
Net* net_create(lq_ctx* ctx, int nlayers);
void net_destroy(Net* n);
int net_layers(const Net* n);
lq_ctx* net_ctx(const Net* n);
void net_set_weights(Net* n, const double* host);  // [L][9][4][4] complex
void net_get_weights(Net* n, double* host);
void net_init_neumann(Net* n, double kappa);
void net_get_grad(Net* n, double* host);            // dL/dconj(W) of the last loss
void net_zero_grad(Net* n);
void net_apply_even(Net* n, void* y_e, const void* x_e, bool adjoint);
void net_apply_even_fast(Net* n, void* y_e, const void* x_e, bool adjoint);  // FP16 inside
double net_loss_grad(Net* n, const void* b, const void* x, int npairs);
void net_adam(Net* n, double lr, double b1, double b2, double eps);
void net_train(Net* n, const void* b, const void* x, int npairs, int epochs, int batch, double lr,
               unsigned seed, double* hist);
// complex BLAS on one-parity fields (elementwise over complex entries)
void caxpy_f32(lq_ctx* ctx, void* y, double cr, double ci, const void* x);        // y += c x
void caxpy_64_32(lq_ctx* ctx, void* y64, double cr, double ci, const void* x32);  // y += c x
void axpby_f32(lq_ctx* ctx, void* out, double a, const void* x, double b, const void* y);
constexpr int MDOT_BLOCKS_MAX = 256;  // partial rows per vector of multidot_f32
// res_host[2i], res_host[2i+1] = <V_i, w> for the nv fields whose device
// pointers are at vdev; part: nv * 256 * 2 doubles, res_dev: 2 nv doubles
void multidot_f32(lq_ctx* ctx, const void* vdev, int nv, const void* w, double* part,
                  double* res_dev, double* res_host);
// w -= sum_i c_i V_i, c_dev: nv complex (double2) on the device
void multiaxpy_f32(lq_ctx* ctx, const void* vdev, int nv, const double* c_dev, void* w);
void mrhs_iterate(lq_ctx* ctx, MRWork* w, int check_every, bool use_graph);
void mrhs_state_upload(lq_ctx* ctx, MRWork* w);
void mrhs_state_download(lq_ctx* ctx, MRWork* w);
double mrhs_iteration_site_bytes(int nrhs);
void mrhs_slot_from_single(lq_ctx* ctx, MRWork* w, void* mfield, int prec, void* single,
                           int r, double a, double b, int single_prec = LQ_F64);
void mrhs_single_from_slot(lq_ctx* ctx, MRWork* w, void* mfield, int prec, void* single64,
                           int r, double a, double b);

// ensemble.hip: uneven batch (member contexts must outlive the batch)
Ensemble* ensemble_create(lq_ctx* const* members, int n);
void ensemble_destroy(Ensemble* e);
void ensemble_tune(Ensemble* e, int inner, const char* cache_path, lq_ensemble_report* rep);
void ensemble_solve(Ensemble* e, void* const* dev_x, const void* const* dev_b, const double* kappa,
                    const double* csw, double tol, const lq_solver_params* params,
                    lq_solve_report* reports, lq_ensemble_report* rep);

inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

// Compulsory bytes per site of one field or table in each precision: a spinor
// (12 complex; FP16 adds its 4-byte scale), a 12-real compressed link, and
// the two Hermitian 6x6 clover blocks (72 reals).
inline double spinor_site_bytes(int prec) {
  return prec == LQ_F64 ? 192.0 : prec == LQ_F32 ? 96.0 : 52.0;
}
inline double link_site_bytes(int prec) { return prec == LQ_F64 ? 96.0 : prec == LQ_F32 ? 48.0 : 24.0; }
inline double clover_site_bytes(int prec) {
  return prec == LQ_F64 ? 576.0 : prec == LQ_F32 ? 288.0 : 144.0;
}
// One even-odd hopping sweep: 8 links, one input and one output spinor per site.
inline double dslash_site_bytes(int prec) {
  return 8 * link_site_bytes(prec) + 2 * spinor_site_bytes(prec);
}

}  // namespace lq
