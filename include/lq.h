/*
 * lq.h -- C ABI of the MI355X (gfx950) Wilson-clover even-odd operator and
 * Krylov solvers.
 *
 * The problem is the one the paper states (section 3, eq. "linear"): solve
 * M phi = b, or the normal equations M^dagger M phi = b, for the Wilson or
 * clover fermion matrix M, a huge sparse complex non-Hermitian matrix, with
 * an iterative method whose cost is dominated by the matrix-vector product
 * (sections 3 and 5).  Section 5 adds the even-odd (Schur complement)
 * reduction, CG on the normal operator, and mixed precision through
 * iterative refinement.  The operator itself is not printed in the paper;
 * the conventions used are:
 *
 *   M = A - kappa H,
 *   (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                        + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)],
 *   A(x) = 1 - csw kappa sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
 *   F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dagger)/(8i) minus its trace/3,
 *     Q_{mu nu} the four mu->nu ordered plaquette leaves at x;
 *   Hermitian chiral-basis gammas: gamma_k = [[0, -i s_k], [i s_k, 0]]
 *     (k = 1,2,3 <-> mu = 0,1,2), gamma_4 = [[0, 1], [1, 0]] (mu = 3),
 *     gamma_5 = diag(1, 1, -1, -1);
 *   links periodic; fermion hops periodic in x, y, z and, when
 *     t_antiperiodic != 0, antiperiodic in t;
 *   parity (x0+x1+x2+x3) mod 2, even = 0;
 *   Schur operator  Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe  on even sites,
 *   bhat_e = b_e + kappa H_eo A_oo^{-1} b_o,
 *   x_o = A_oo^{-1} (b_o + kappa H_oe x_e).
 *
 * Host layouts (complex128 = two doubles, real then imaginary):
 *   site index i = ((x3*Lz + x2)*Ly + x1)*Lx + x0 (x fastest, t = x3);
 *   gauge  U[i][mu][a][b], U_mu(x) the link from x to x+mu;
 *   spinor psi[i][spin][colour];
 *   a half-lattice array lists the V/2 sites of one parity in increasing i;
 *   with nrhs > 1 the right-hand side index is slowest: psi[r][site][s][a].
 *
 * Device fields are opaque byte buffers of lq_field_bytes() bytes, owned
 * by the caller (any device allocation, 256-byte aligned).  Their inner
 * layout is private to the library (site-blocked, 64 sites per block;
 * FP64 component-major inside a block, FP32 and FP16 in 16-byte chunks of
 * components; FP16 fields carry one FP32 scale per site).
 *
 * Every call returns an lq_status; no C++ exception crosses this boundary.
 * On failure a message is kept in the context (lq_last_error).  All device
 * work is issued on the stream given to lq_create; calls that return host
 * data synchronise that stream.  A context must not be used from two
 * threads at once; separate contexts are independent.
 */
#ifndef LQ_H
#define LQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lq_ctx lq_ctx;

typedef enum {
  LQ_OK = 0,
  LQ_EINVAL = -1,   /* bad argument (sizes, parity, precision, null pointer, not SU(3)) */
  LQ_ENOMEM = -2,   /* device or host allocation failed */
  LQ_EHIP = -3,     /* a HIP runtime call failed */
  LQ_ENOCONV = -4,  /* solver did not reach the tolerance; report filled */
  LQ_ESTATE = -5,   /* call out of order (no gauge field, no clover term) */
  LQ_ENAN = -6      /* NaN or Inf met in a reduction; report filled */
} lq_status;

/* LQ_F16X: FP16 with the right-hand sides of one parity interleaved per site
 * (up to 16 RHS in one field; the layout of the matrix-core multi-RHS
 * operator).  Accepted by lq_field_bytes, lq_spinor_to_device/_to_host
 * (parity EVEN or ODD), lq_dslash and lq_schur. */
typedef enum { LQ_F64 = 0, LQ_F32 = 1, LQ_F16 = 2, LQ_F16X = 3 } lq_prec;
typedef enum { LQ_EVEN = 0, LQ_ODD = 1, LQ_FULL = 2 } lq_parity;
typedef enum {
  LQ_CGNR = 0,         /* CG on Mhat^dagger Mhat (plain FP64 when inner_prec = F64) */
  LQ_BICGSTAB = 1,     /* BiCGStab on Mhat */
  LQ_FGMRES_NET = 2,   /* FGMRES(m) on Mhat, learned preconditioner on the right */
  LQ_FCG_NET = 3       /* flexible CG on Mhat^dagger Mhat with N_e N_e^dagger */
} lq_solver;

/* Solver parameters.  Zero-initialise and set what you need; zeros select
 * the defaults given per field. */
typedef struct {
  int solver;            /* lq_solver, default LQ_CGNR */
  int inner_prec;        /* lq_prec of the inner iteration: F64 = plain solve,
                            F32/F16 = mixed precision with FP64 reliable updates */
  int maxiter;           /* total inner iterations, default 20000 */
  double delta;          /* reliable-update trigger ||r|| < delta * max ||r||, default 0.1
                            (0.03 for batched = 1) */
  int restart;           /* FGMRES restart length m, default 32 */
  int check_every;       /* iterations per captured graph replay, default 8 */
  int use_graph;         /* 1 (default when 0 is given: 1) replay captured iterations;
                            -1 launch each kernel directly */
  int fault_inject;      /* tests only: 1 = force the inner solve to stagnate */
  int profile;           /* 1: time every inner-iteration kernel with HIP events (no graph) */
  int batched;           /* 1: solve all nrhs (<= 16) together through the multi-RHS operator
                            (CGNR, inner_prec F16): one operator application serves every RHS,
                            independent CG recurrences; 2: the same operator in block CG, one
                            Krylov space shared by all RHS (O'Leary's block conjugate gradient,
                            rank-revealing search block, reliable updates per RHS) */
  int deflate;           /* LQ_FGMRES_NET: k > 0 deflated vectors (k < restart, at most 32)
                            kept across restarts (FGMRES-DR, section 7 of the paper); restart
                            then defaults to 70 */
  const void* dev_xref;  /* optional reference solution(s) on the device (full-lattice FP64
                            fields laid out as dev_x, nrhs of them): the report then gives
                            ||x - xref|| / ||xref|| per right-hand side (ref_error) */
} lq_solver_params;

/* Kernels of one inner CG iteration, in launch order (report index). */
enum {
  LQ_K_HOP_OE = 0,   /* t = A_oo^-1 H_oe p */
  LQ_K_HOP_EO = 1,   /* q = A_ee p - kappa^2 H_eo t, |q|^2 */
  LQ_K_HOPD_OE = 2,  /* t = A_oo^-1 H^+_oe q */
  LQ_K_UPDATE = 3,   /* A_ee q - kappa^2 H^+_eo t fused with x, r, rt updates, |r|^2 */
  LQ_K_PUPDATE = 4,  /* p = r + beta p */
  LQ_NK = 5
};

typedef struct {
  int iterations;          /* inner iterations (all restarts, all RHS max) */
  int reliable_updates;    /* FP64 true-residual recomputations */
  int fallback;            /* 1 if the plain FP64 solver had to finish the solve */
  int dslash_calls;        /* hopping-term sweeps issued (per RHS) */
  double true_residual;    /* ||b - M x|| / ||b|| of the full system, FP64 */
  double schur_residual;   /* ||bhat - Mhat x_e|| / ||bhat||, FP64 */
  double seconds;          /* wall time of the solve inside the library */
  double bytes;            /* algorithmic (compulsory) bytes of every kernel launched */
  double kernel_ms[LQ_NK];      /* profile = 1: summed durations per iteration kernel */
  double kernel_bytes[LQ_NK];   /* algorithmic bytes of one launch of each kernel */
  int kernel_calls[LQ_NK];      /* profile = 1: launches timed per kernel */
  double ref_error;        /* ||x - xref|| / ||xref|| when params->dev_xref is given, else -1 */
} lq_solve_report;

/* Context: owns device copies of the gauge field (12-real compressed, FP64,
 * FP32 and FP16), the clover term and solver work space.  dims = {Lx, Ly,
 * Lz, Lt}, each even and >= 2.  stream: a hipStream_t (NULL = default). */
lq_status lq_create(const int dims[4], int t_antiperiodic, void* hip_stream, lq_ctx** out);
void lq_destroy(lq_ctx* ctx);
/* Last error message of ctx (or of the last failed lq_create when ctx is NULL);
 * valid until the next call on ctx. */
const char* lq_last_error(const lq_ctx* ctx);
/* Bytes of a device field: parity EVEN/ODD = V/2 sites, FULL = both halves. */
size_t lq_field_bytes(const lq_ctx* ctx, int parity, int prec, int nrhs);
/* Local volume V and padded half volume (sites per parity rounded up to 64). */
int64_t lq_volume(const lq_ctx* ctx);

/* Gauge field upload and 12-real compression (rows 0 and 1 kept, row 2 =
 * conj(row0 x row1) rebuilt in the kernels).  host_U: V*4*9 complex128,
 * caller-owned, read during the call.  Fails with LQ_EINVAL unless every
 * link is unitary with det 1 to 1e-12. */
lq_status lq_upload_gauge(lq_ctx* ctx, const double* host_U);

/* Build the clover term for (kappa, csw) on the GPU in FP64 from the FP64
 * links: A on both parities, A^{-1} on both parities, and FP32/FP16 copies
 * of A_ee and A_oo^{-1}.  csw = 0 gives A = 1 (plain Wilson). */
lq_status lq_set_clover(lq_ctx* ctx, double kappa, double csw);

/* Host canonical spinor(s) -> device field of precision prec (FP16: per-site
 * scale = max |component| over the 24 reals, components stored as
 * fp16(value/scale)), and back.  parity EVEN/ODD: host holds V/2 sites;
 * FULL: host holds V sites.  Synchronous with respect to host memory. */
lq_status lq_spinor_to_device(lq_ctx* ctx, void* dev, const double* host, int parity,
                              int prec, int nrhs);
lq_status lq_spinor_to_host(lq_ctx* ctx, double* host, const void* dev, int parity,
                            int prec, int nrhs);

/* Even-odd hopping term: out = H_eo in (out_parity EVEN, in odd) or H_oe in
 * (out_parity ODD, in even); dagger != 0 applies the blocks of H^dagger.
 * Both fields of precision prec; asynchronous on the context stream. */
lq_status lq_dslash(lq_ctx* ctx, void* dev_out, const void* dev_in, int out_parity,
                    int dagger, int prec, int nrhs);

/* out = A_pp in or A_pp^{-1} in on one parity.  F64 supports both parities
 * and both forms; F32/F16 support A_ee and A_oo^{-1}. */
lq_status lq_clover_apply(lq_ctx* ctx, void* dev_out, const void* dev_in, int parity,
                          int inverse, int prec, int nrhs);

/* Schur operator on even fields: out = Mhat in (dagger = 0) or Mhat^dagger in.
 * Needs lq_set_clover.  dev_tmp: caller buffer of lq_field_bytes(ODD, prec, nrhs). */
lq_status lq_schur(lq_ctx* ctx, void* dev_out, const void* dev_in, void* dev_tmp, int dagger,
                   int prec, int nrhs);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: lq_schur
 * without dev_tmp.  The odd-parity intermediate A_oo^-1 H_oe in lives in a
 * static device array of LQ_SCRATCH_BYTES bytes that every GPU the library
 * runs on holds until the process ends; the call allocates nothing (the
 * array's address on a device is resolved by lq_create).  prec: LQ_F64,
 * LQ_F32 or LQ_F16 (LQ_EINVAL for LQ_F16X, whose operator tables the library
 * allocates); LQ_EINVAL when one odd field of the lattice in prec exceeds
 * LQ_SCRATCH_BYTES (lq_field_bytes(ctx, LQ_ODD, prec, 1) > LQ_SCRATCH_BYTES;
 * e.g. a 32^3x64 lattice fits in FP16 only).  nrhs fields run one after
 * another.  Every call on one GPU shares the array, which keeps the last
 * call's contents: calls that overlap in time on one GPU (other streams,
 * other threads, other contexts) race, and the caller must serialise them.
 * Results equal lq_schur's. */
#define LQ_SCRATCH_BYTES ((size_t)64 << 20)
lq_status lq_schur_noalloc(lq_ctx* ctx, void* dev_out, const void* dev_in, int dagger, int prec,
                           int nrhs);

/* ------------------------------------------------------------------------
 * Tiling and its tuner.  Each parity's sites are numbered inside 4-D tiles
 * (every extent an even divisor of the lattice extent; the tile with the
 * least surface per volume among those of at most `tile_sites` sites of one
 * parity): within a tile the y, z and t neighbours of 64 consecutive sites
 * are 64 consecutive sites, and the tile size sets how far a neighbour across
 * it lies in memory.  The 12-RHS fields have their own, smaller tiles.
 * Defaults: 65536 and 2048 sites (measured on MI355X at 32^3x64).
 * ------------------------------------------------------------------------ */

/* Change the largest tile of the single-RHS numbering (tile_sites) and of
 * the multi-RHS numbering (mr_tile_sites); 0 keeps the current one, other
 * values below 64 are LQ_EINVAL.  Only before the gauge field is uploaded
 * and before any solver work space exists (else LQ_ESTATE): every field is
 * laid out in this numbering. */
lq_status lq_set_tiling(lq_ctx* ctx, int64_t tile_sites, int64_t mr_tile_sites);
/* The tile extents in use (either pointer may be NULL). */
lq_status lq_get_tiling(const lq_ctx* ctx, int tiles[4], int mr_tiles[4]);

#define LQ_TUNE_MAX 8
typedef struct {
  int ncand;                        /* candidates measured (distinct tilings) */
  int64_t target[LQ_TUNE_MAX];      /* their largest tile, sites of one parity */
  int tiles[LQ_TUNE_MAX][4];        /* their tile extents */
  double us[LQ_TUNE_MAX];           /* time of one Schur application (0: unknown) */
  int best;                         /* index of the chosen candidate */
  int from_cache;                   /* 1: the choice was read from the cache file */
} lq_tune_report;

/* Choose the tile for a lattice of `dims` (t_antiperiodic as lq_create):
 * for prec LQ_F64 / LQ_F32 / LQ_F16 with nrhs = 1 the single-RHS tile
 * (candidates 4096, 16384, 65536, 262144 sites and one tile for the whole
 * lattice), for LQ_F16X with nrhs 1..16 the multi-RHS tile (512, 1024, 2048,
 * 8192, 32768), candidates giving the same tiling measured once.  Each is
 * timed on a scratch context with unit links and the clover term of
 * kappa 0.135, csw 1 (the kernels' work does not depend on the values): 20
 * applications of the Schur operator (lq_schur) after 3 warm-ups, on a
 * stream of its own, HIP events around them.  The fastest is the choice.
 * With cache_path (may be NULL) the choice is first looked up in that JSON
 * file under the key "<arch>:<precision>:nrhs<n>:<dims>" and written there
 * after a measurement (other keys are kept).  Apply it with lq_set_tiling
 * on a new context.  Needs a GPU and several GB of free device memory for
 * the scratch contexts.  Errors: lq_tune_last_error(). */
lq_status lq_tune_tiles(const int dims[4], int t_antiperiodic, int prec, int nrhs,
                        const char* cache_path, lq_tune_report* rep);
const char* lq_tune_last_error(void);

/* Measurement reference: copy `bytes` (a multiple of 16; both pointers
 * 16-byte aligned, else LQ_EINVAL) from src to dst with 16-byte loads and
 * stores per lane, asynchronously on `stream` (a hipStream_t, NULL =
 * default).  Its rate, read plus write, is the achievable HBM bandwidth the
 * hopping term is compared with; it needs no context. */
lq_status lq_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Fused site-local lattice expressions (the data-parallel expressions of the
 * QDP++ library that section 4 of the paper ports; its worked example is
 * the SU(3) array product U_x = V_x W_x of section 3, eq. su3vecmul).  Each
 * call is one kernel that reads every operand element once and writes the
 * result once, whatever the length of the expression.  Arrays hold n site
 * elements (complex 3x3 colour matrices, or 4 x 3 spinors) in the
 * library's blocked device layout (lq_site_array_bytes bytes), FP64 or FP32;
 * host arrays are element-major complex128 (matrix row-major; spinor
 * spin-major).  The output may be one of the inputs (each element is read
 * before it is written).  Asynchronous on `stream` (a hipStream_t) except
 * the transfers, which synchronise it.  LQ_EINVAL on bad arguments.
 * ------------------------------------------------------------------------ */
enum { LQ_SITE_SU3 = 0, LQ_SITE_SPINOR = 1 };
enum {
  LQ_SU3_VW = 0,      /* U = V W (eq. su3vecmul) */
  LQ_SU3_VWDAG = 1,   /* U = V W^dagger */
  LQ_SU3_VDAGW = 2,   /* U = V^dagger W */
  LQ_SU3_VWX = 3      /* U = V W X, one fused pass */
};
size_t lq_site_array_bytes(int64_t n, int kind, int prec);
lq_status lq_site_array_to_device(void* dev, const double* host, int64_t n, int kind, int prec,
                                  void* stream);
lq_status lq_site_array_to_host(double* host, const void* dev, int64_t n, int kind, int prec,
                                void* stream);
lq_status lq_su3_mul(void* dev_u, const void* dev_v, const void* dev_w, const void* dev_x,
                     int64_t n, int form, int prec, void* stream);
/* out_x = U_x in_x (U^dagger when adjoint_u != 0) on every spin of each spinor */
lq_status lq_su3_spinor_mul(void* dev_out, const void* dev_u, const void* dev_in, int64_t n,
                            int adjoint_u, int prec, void* stream);

/* Global reductions on a device field (FP64 accumulation, fixed tree order):
 * out[0] = sum |a|^2; dot: out[0] + i out[1] = sum conj(a) b. */
lq_status lq_norm2(lq_ctx* ctx, double* out, const void* dev_a, int parity, int prec);
lq_status lq_dot(lq_ctx* ctx, double* out, const void* dev_a, const void* dev_b, int parity,
                 int prec);

/* Solve M x = b on the full lattice for nrhs right-hand sides with the
 * clover term of (kappa, csw) (rebuilt if these differ from the current
 * ones).  Stops when the FP64 true residual ||b - M x|| / ||b|| <= tol for
 * every RHS.  host_b, host_x: nrhs * V * 12 complex128.  report: nrhs
 * entries (may be NULL).  Returns LQ_ENOCONV when maxiter is reached. */
lq_status lq_solve(lq_ctx* ctx, double* host_x, const double* host_b, int nrhs, double kappa,
                   double csw, double tol, const lq_solver_params* params,
                   lq_solve_report* report);

/* The same solve on device-resident fields: dev_b and dev_x are full-lattice
 * FP64 fields (lq_field_bytes(ctx, LQ_FULL, LQ_F64, nrhs) bytes each, as
 * written by lq_spinor_to_device with parity LQ_FULL), caller-owned and
 * distinct.  dev_x is overwritten with the solution; no host transfer of
 * b or x takes place.  The call returns after the solve has finished. */
lq_status lq_solve_device(lq_ctx* ctx, void* dev_x, const void* dev_b, int nrhs, double kappa,
                          double csw, double tol, const lq_solver_params* params,
                          lq_solve_report* report);

/* ------------------------------------------------------------------------
 * SAP preconditioner and FGCR: the solver of section 5 of the paper.
 * The lattice is cut into non-overlapping blocks coloured like a
 * checkerboard.  One application K of the Schwarz alternating procedure runs
 * ncycles cycles from zero.  A cycle takes, for each colour in turn (colour
 * 0 = even sum of block coordinates first), nmr minimal-residual steps on
 * the Wilson-clover equation restricted to every block of that colour
 * (Dirichlet boundary conditions: hops leaving a block are dropped), then
 * recomputes the residual.  K is not a fixed matrix, so it serves as the
 * right preconditioner of a flexible GCR (FGCR), restarted every `restart`
 * steps with the residual recomputed in FP64 and the FP32 correction added
 * to the FP64 solution (iterative refinement).  Block solves and the inner
 * FGCR run in FP32. */
typedef struct {
  int block[4];  /* block extents (x, y, z, t): each divides the lattice extent an even
                    number of times; at most 512 sites per block */
  int ncycles;   /* SAP cycles per application (0: 5) */
  int nmr;       /* MR steps per block solve (0: 4) */
  int restart;   /* FGCR steps between FP64 restarts (0: 16, at most 64); with deflate > 0
                    the Krylov dimension m of FGMRES-DR including the deflated vectors
                    (0: 70, at most 128) */
  int maxiter;   /* FGCR steps in all (0: 2000) */
  int deflate;   /* 0: FGCR.  k > 0: FGMRES with deflated restarting (section 7 of the
                    paper): k harmonic Ritz vectors (k < m, at most 32) of the Arnoldi
                    matrix are kept across each restart; the residual is recomputed in FP64
                    at every restart */
  int block_fp16; /* 0: the block solves apply the operator with FP32 links (copied to
                     LDS) and FP32 clover blocks (read from HBM at every MR step).  1: with
                     FP16 links and clover blocks, staged in LDS beside the FP32 residual
                     once per block (arithmetic FP32); LQ_EINVAL when they do not fit
                     (at most 512 sites per block as always; 8x4x4x4 fits).  The
                     preconditioner then differs from the FP32 one by the FP16 rounding of
                     the operator, which the flexible outer solver absorbs */
  int block_eo;   /* 1 (with block_fp16 = 1 and an even x extent of the blocks): MR on the
                     even-odd reduced block operator A_ee - kappa^2 H_eo A_oo^-1 H_oe
                     (block-restricted hopping term) from the source r_e + kappa H_eo
                     A_oo^-1 r_o, then d_o = A_oo^-1 (r_o + kappa H_oe d_e): the block
                     solve the paper's performance model counts (section 5, eq.
                     sapmodel).  0: MR on the block operator itself */
} lq_sap_params;

/* dev_out = K dev_in on full-lattice FP32 fields (lq_field_bytes(ctx,
 * LQ_FULL, LQ_F32, 1) bytes; distinct buffers), with the clover term of the
 * last lq_set_clover or solve.  Runs on the context's stream; LQ_EINVAL for
 * a block layout the lattice does not admit, LQ_ESTATE without gauge field
 * or clover term. */
lq_status lq_sap_apply(lq_ctx* ctx, void* dev_out, const void* dev_in,
                       const lq_sap_params* params);

/* Solve M x = b by SAP-preconditioned FGCR (or FGMRES-DR when
 * params->deflate > 0) to ||b - M x|| <= tol ||b|| (FP64 true residual).  dev_b, dev_x: full-lattice FP64 fields as for
 * lq_solve_device (distinct; dev_x is overwritten).  report (may be NULL):
 * iterations = FGCR steps, reliable_updates = FP64 restarts, true_residual.
 * LQ_ENOCONV when maxiter steps do not reach tol, or when restarts stop
 * reducing the residual (five FGCR restarts, or three FGMRES-DR restarts, in
 * a row without halving it). */
lq_status lq_solve_sap(lq_ctx* ctx, void* dev_x, const void* dev_b, double kappa, double csw,
                       double tol, const lq_sap_params* params, lq_solve_report* report);

/* ------------------------------------------------------------------------
 * Learned preconditioner.  The paper's solvers are flexible Krylov methods
 * (its FGCR, equivalent to FGMRES, around a preconditioner that is itself an
 * iteration: section 5), which admit a preconditioner that is not a fixed
 * matrix.  This library supplies as such a preconditioner a linear,
 * gauge-covariant net of nlayers layers on full-lattice spinors,
 *
 *   psi_{l+1}(x) = W0 psi_l(x) + sum_mu [ Wp_mu U_mu(x) psi_l(x+mu)
 *                                        + Wm_mu U_mu(x-mu)^+ psi_l(x-mu) ],
 *
 * with complex 4x4 spin matrices W (colour-blind) and the fermion boundary
 * phase of the hopping term.  On the even-odd system it acts as
 * N_e = P_e N E_e (embed an even field with zeros on the odd sites, apply,
 * keep the even sites).  Weights on the host: double[nlayers][9][4][4][2]
 * (re, im), index k = 0: W0, 1 + 2 mu: Wp_mu, 2 + 2 mu: Wm_mu, matrix row =
 * output spin.  Device fields of the net calls are LQ_F32 even fields
 * (lq_field_bytes(ctx, LQ_EVEN, LQ_F32, n)), caller-owned.  A net holds FP32
 * weights, Adam moments, activations of one sample and its gradient; it
 * uses the gauge field its context holds at each call.  Errors are reported
 * through the context's lq_last_error.
 * ------------------------------------------------------------------------ */
typedef struct lq_net lq_net;

/* A net of nlayers (1..16) layers with zero weights; needs a gauge field. */
lq_status lq_net_create(lq_ctx* ctx, int nlayers, lq_net** out);
void lq_net_destroy(lq_net* net);

/* Copy weights in (EINVAL on non-finite values; resets the Adam state) or out. */
lq_status lq_net_set_weights(lq_net* net, const double* host_w);
lq_status lq_net_get_weights(lq_net* net, double* host_w);

/* The Neumann start of training: W0 = 1, Wp_mu = -(kappa / w_l)(1 - gamma_mu),
 * Wm_mu = -(kappa / w_l)(1 + gamma_mu) with w_l = exp(2 pi i (l+1) / (nlayers+1)),
 * which makes the net the truncated series sum_{n <= nlayers} (kappa H)^n of
 * the hopping term H (gamma matrices of the chiral basis of lq_dslash). */
lq_status lq_net_init_neumann(lq_net* net, double kappa);

/* dev_out = N_e dev_in (distinct buffers); mode is a sum of flags:
 * LQ_NET_ADJOINT applies N_e^+; LQ_NET_FP16 computes with FP16 links, FP16
 * weights and FP16 activations (per-site FP32 scales) and FP32 accumulation
 * (spin mixing on the matrix cores), the form the solvers use; its result
 * agrees with the FP32 form to a few 1e-4 relative.  Otherwise FP32 links,
 * weights and activations. */
enum { LQ_NET_ADJOINT = 1, LQ_NET_FP16 = 2 };
lq_status lq_net_apply(lq_net* net, void* dev_out, const void* dev_in, int mode);

/* Training loss over npairs (source b_i, target x_i) pairs, each a set of
 * npairs consecutive even fields:  loss = mean_i ||N_e b_i - x_i||^2 / ||x_i||^2.
 * Its gradient dL/dconj(W) (Wirtinger convention; the real gradient is
 * 2 Re, 2 Im of it) replaces the net's stored gradient and, if host_grad is
 * not NULL, is copied there (layout of the weights). */
lq_status lq_net_loss_grad(lq_net* net, const void* dev_b, const void* dev_x, int npairs,
                           double* loss, double* host_grad);

/* One Adam step on the real parameters (Re W, Im W) with the stored
 * gradient, which is then cleared. */
lq_status lq_net_adam_step(lq_net* net, double lr, double beta1, double beta2, double eps);

/* epochs of Adam (beta = 0.9, 0.999; eps = 1e-8) over the pairs in batches of
 * `batch` drawn by a random permutation per epoch; loss_history (may be
 * NULL) receives the mean loss of each epoch.  The permutations come from a
 * generator the net keeps: seed != 0 restarts it from that seed, seed = 0
 * continues from its current state (after lq_net_load: the saved one). */
lq_status lq_net_train(lq_net* net, const void* dev_b, const void* dev_x, int npairs, int epochs,
                       int batch, double lr, unsigned seed, double* loss_history);

/* Checkpoint of the training state: the FP32 weights, both Adam moment
 * arrays, the Adam step count and the shuffle generator's state, in a file
 * that starts with one line of JSON (format "lq-net-checkpoint", version 1,
 * layers, adam_step, shuffle_state, bytes_per_array) followed by the three
 * arrays (float32 (re, im) pairs, [layers][9][4][4], little endian).  Loading
 * restores them exactly (training continued after lq_net_load with seed 0
 * repeats uninterrupted training step for step) and clears the stored
 * gradient.  LQ_EINVAL on an unreadable, malformed or truncated file, or one
 * of another layer count. */
lq_status lq_net_save(lq_net* net, const char* path);
lq_status lq_net_load(lq_net* net, const char* path);

/* lq_solve with a learned-preconditioner solver: params->solver =
 * LQ_FGMRES_NET (FGMRES(restart) on Mhat, right preconditioner N_e) or
 * LQ_FCG_NET (flexible CG on Mhat^+ Mhat with N_e N_e^+).  Inner cycles in
 * FP32, restarted from the FP64 Schur residual; when the flexible solver
 * stagnates, breaks down or exhausts maxiter, the plain mixed CG finishes
 * the solve and report->fallback is set.  The net must belong to ctx. */
lq_status lq_solve_net(lq_ctx* ctx, lq_net* net, double* host_x, const double* host_b, int nrhs,
                       double kappa, double csw, double tol, const lq_solver_params* params,
                       lq_solve_report* report);

/* ------------------------------------------------------------------------
 * Uneven batch.  Independent solves of M x = b (the even-odd CG of lq_solve
 * with reliable updates, section 5) on lattices of different extents and
 * hopping parameters, one right-hand side each, advanced together: every
 * stage of an iteration is one kernel launch over the site tiles of all
 * members still iterating, the members' scalars stay on the device, the
 * FP64 reliable updates are batched launches inside the iteration, and
 * check_every iterations are replayed from a captured graph between host
 * polls.  Finished members drop out of the tile list.  Members that break
 * down or stagnate are finished by the FP64 CG of their own context
 * (report fallback = 1).
 *
 * Members are distinct contexts of one device with a gauge field; they must
 * outlive the batch and not be used by other calls while it solves.  The
 * batch launches on a stream of its own after synchronising each member's
 * stream; the call returns when every member is finished.
 * ------------------------------------------------------------------------ */
typedef struct lq_ensemble lq_ensemble;

typedef struct {
  int tile_sites;       /* sites per workgroup of the iteration kernels (64, 128, 256) */
  int tile_from_cache;  /* 1: the tile was read from the cache file */
  double tune_ms[3];    /* measured time of one iteration's operator and vector kernels
                           for 64, 128 and 256 sites per workgroup (0: not measured) */
  int graph_captures;   /* graphs captured during the solve */
  int replays;          /* graph replays, each followed by one host poll */
  int iterations;       /* inner iterations of the longest member */
  double seconds;       /* wall time of the whole solve */
  double bytes;         /* algorithmic bytes of all members' kernels */
} lq_ensemble_report;

/* A batch of n (1..64) member contexts.  On failure *out is NULL and
 * lq_ensemble_last_error(NULL) holds the message. */
lq_status lq_ensemble_create(lq_ctx* const* members, int n, lq_ensemble** out);
void lq_ensemble_destroy(lq_ensemble* e);
const char* lq_ensemble_last_error(const lq_ensemble* e);

/* Choose the tile shape for inner precision inner_prec (LQ_F64, LQ_F32 or
 * LQ_F16): from the batch's memory, else from the JSON file cache_path (may
 * be NULL), else by timing every candidate on the members (which need their
 * clover term, lq_set_clover); a measured choice is written to cache_path.
 * The cache key is the GPU architecture, the precision, nrhs = 1 and the
 * members' extents in order.  rep (may be NULL) receives the tile fields. */
lq_status lq_ensemble_tune(lq_ensemble* e, int inner_prec, const char* cache_path,
                           lq_ensemble_report* rep);

/* Solve member j's system with (kappa[j], csw[j]) on full-lattice FP64
 * device fields dev_b[j] -> dev_x[j] (as lq_solve_device; caller-owned,
 * distinct), to the FP64 true residual tol for every member.  params: solver
 * LQ_CGNR, inner_prec, maxiter, delta, check_every, use_graph as for
 * lq_solve (batched and profile must be 0; fault_inject = 1, for tests, makes the
 * members of even index withhold their inner corrections so that they stagnate
 * and fall back).  Tunes on first use
 * of a precision (lq_ensemble_tune without a file).  reports: n entries (may
 * be NULL; seconds = whole batch); rep may be NULL.  Returns LQ_ENOCONV when
 * a member did not converge, with the reports filled. */
lq_status lq_ensemble_solve(lq_ensemble* e, void* const* dev_x, const void* const* dev_b,
                            const double* kappa, const double* csw, double tol,
                            const lq_solver_params* params, lq_solve_report* reports,
                            lq_ensemble_report* rep);

#ifdef __cplusplus
}
#endif

#endif /* LQ_H */
