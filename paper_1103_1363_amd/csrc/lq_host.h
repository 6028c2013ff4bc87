// Host side of the lq library: the context, the declarations of every
// source file's functions and the algorithmic byte counts.  Holds no device
// code (the kernels' code follows from lq_internal.h and the headers of the
// kernels).
#pragma once

#include <functional>

#include "lq_internal.h"

namespace lq {

// ---------------------------------------------------------------- context
struct Clover {
  // FP64: A and A^{-1} for both parities; lower precisions: A_ee and A_oo^{-1}
  void* a64[2] = {nullptr, nullptr};
  void* ainv64[2] = {nullptr, nullptr};
  void* a_ee[3] = {nullptr, nullptr, nullptr};
  void* ainv_oo[3] = {nullptr, nullptr, nullptr};
  double kappa = 0, csw = 0;
  bool valid = false;
  // Incremented by every build: caches derived from the clover tables (the
  // SAP solver's FP32 copy) compare it instead of (kappa, csw), which stay
  // equal when a new gauge field is uploaded.
  uint64_t gen = 0;
};

struct Work;    // solver work space (solver.hip)
struct MRWork;  // batched multi-RHS solver work space (mrhs.hip)
struct Net;     // learned preconditioner (net.hip)
struct Ensemble;  // uneven batch of independent solves (ensemble.hip)
struct Sap;       // SAP preconditioner state (sap.hip)
struct KrylovWork;  // deflated FGMRES work space (krylov.hip)
struct BlockWork;   // block CG work space (solver.hip)

}  // namespace lq

struct lq_ctx {
  lq::Geo geo;
  // Site numbering of the multi-RHS fields and tables: the same lattice in
  // smaller tiles.  A site's nrhs spinors sit together (hundreds of bytes),
  // so the neighbours across a tile must stay within the reach of L2.
  lq::Geo mr_geo;
  int dims[4];
  int64_t V;
  int device = 0;                 // HIP device current at lq_create
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
  lq::Sap* sap = nullptr;   // SAP preconditioner state (lazy)
  lq::KrylovWork* kwork = nullptr;  // deflated FGMRES work space (lazy)
  lq::BlockWork* bwork = nullptr;   // block CG work space (lazy)
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
void upload_unit_gauge(lq_ctx* ctx);  // U = 1 everywhere (timing only)
int64_t tile_target();
int64_t mr_tile_target();
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

// sap.hip: SAP preconditioner on full FP32 fields, and FGCR around it on
// full FP64 fields (returns whether ||b - M x|| <= tol ||b||)
void sap_apply(lq_ctx* ctx, void* out, const void* in, const lq_sap_params& q);
bool solve_sap(lq_ctx* ctx, void* x, const void* b, double tol, const lq_sap_params& q,
               lq_solve_report* rep);
bool solve_sap_dr(lq_ctx* ctx, void* x, const void* b, double tol, const lq_sap_params& q,
                  lq_solve_report* rep);  // FGMRES-DR (q.deflate > 0)
void sap_destroy(Sap* sp);
void free_clover(lq_ctx* ctx);

// noalloc.hip: the scratch array's device address, resolved once per
// device (with that device current); the Schur operator that uses it
void noalloc_init(int device);
void schur_noalloc(lq_ctx* ctx, void* out, const void* in, int dagger, int prec, int nrhs);


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
void free_block_work(lq_ctx* ctx);
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

// krylov.hip: FGMRES with deflated restarting on FP32 fields of n complex
// entries (one parity: halves = 1; a full field, even half then odd half:
// halves = 2), FP64 residual and solution.  The callbacks apply the
// preconditioner z = K v and the operator w = A z (FP32 fields), and
// recompute r64 = b - A x64 in FP64 returning |r64|^2; they count their own
// operator sweeps.
struct KrylovSpace {
  int64_t n = 0;
  int halves = 1;
  int64_t vh = 0;  // sites per parity (the rest of each half is padding)
  void* x64 = nullptr;
  void* r64 = nullptr;
  std::function<void(void*, const void*)> precond, op;
  std::function<double()> residual64;
};
// Returns true when |r64| <= target; false on maxiter (breakdown = false) or
// on a breakdown or three restarts without halving the residual
// (breakdown = true).  Counts iterations (preconditioned steps) and
// restarts (as reliable updates) in t.
bool fgmres_dr(lq_ctx* ctx, const KrylovSpace& S, int m, int k, double target, int maxiter,
               SolveTally& t, bool& breakdown);
void free_krylov(lq_ctx* ctx);
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
void mrhs_normal(lq_ctx* ctx, void* q32, const void* p, void* t, void* q1, int nrhs);
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
void net_save(Net* n, const char* path);
void net_load(Net* n, const char* path);
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
