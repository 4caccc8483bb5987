/*
 * libqcd: Wilson-Dirac solver with FP16/FP32 inner BiCGStab and FP64
 * iterative refinement, for AMD Instinct MI355X (gfx950).
 *
 * Method: Kanamori et al., "Mixed precision solvers with half-precision
 * floating point numbers for Lattice QCD on A64FX processor" (SCA/HPCAsia
 * 2026 Workshops).  The operator is the Wilson matrix of eq. (1), the inner
 * solver the rescaled BiCGStab of Alg. 4 / Alg. 5, the outer solver the
 * rescaled iterative refinement of Alg. 3 (Alg. 2 as a special case).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: extents dims[4] = {Lx, Ly, Lz, Lt}, each even and >= 2; periodic
 *   boundaries in all four directions.  Site index s = x + Lx*(y + Ly*(z + Lz*t)).
 * Canonical layouts (device memory, complex128 = two doubles re, im):
 *   gauge field U[s][mu][a][b], mu = 0..3 for x, y, z, t; U_mu(x) is the link
 *   from x to x + mu (Sec. 2, first paragraph);
 *   spinor field psi[s][spin][colour] (12 complex per site).
 * Native layout: the library's own device layout (checkerboarded, blocks of
 *   64 sites, component-major within a block) in a chosen precision; sizes
 *   from qcd_spinor_bytes().  Only pass native buffers produced by this
 *   library for the same gauge handle.
 * Gamma matrices: the Dirac basis whose gamma_1 is the one printed in Sec. 2
 *   (gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = diag(1,1,-1,-1)).
 * Pointers named *_dev are device pointers; the caller owns all device
 *   memory passed in.  Canonical complex128 fields must be 16-byte aligned
 *   (QCD_ERR_ARG otherwise).  `stream` is a hipStream_t (NULL = default stream).
 * Several right-hand sides: calls taking nrhs (1..64) expect nrhs fields
 *   back to back (canonical: [rhs][site][spin][colour]; native: nrhs native
 *   fields of qcd_spinor_bytes() each); per-right-hand-side outputs (norms,
 *   info) are arrays of nrhs entries.
 *   Entry points that return solver results synchronise with `stream`.
 * Errors: a negative status; qcd_last_error() gives a message (per thread).
 *   No C++ exception crosses this interface.
 */
#ifndef QCD_H
#define QCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QCD_OK = 0,
  QCD_NOT_CONVERGED = 1,   /* warning: outputs valid, tolerance not reached in max iterations */
  QCD_ERR_ARG = -1,        /* invalid argument (null pointer, odd extent, kappa <= 0, ...) */
  QCD_ERR_HIP = -2,        /* a HIP runtime call failed */
  QCD_ERR_NONFINITE = -3,  /* a solver scalar became Inf/NaN (e.g. FP16 overflow) */
  QCD_ERR_WORKSPACE = -4,  /* caller workspace smaller than qcd_workspace_bytes() */
  QCD_ERR_UNSUPPORTED = -5,
  QCD_ERR_BREAKDOWN = -6   /* BiCGStab breakdown: rho = (r*, r) = 0 or (r*, A p) = 0 */
} qcd_status;

/* Storage precisions of fields and links (Table 1).  FP16 and BF16 store a
 * complex number as two 16-bit halves of one 32-bit word.  Arithmetic on FP16
 * storage: in the Wilson operator the spin projection is one binary16 add per
 * component (as the paper's FP16 arithmetic, Sec. 5), row 2 of a two-row
 * link is rebuilt with binary16 multiplies and fused multiply-adds, and each
 * link product is a pair of exact binary16 products summed in FP32
 * (v_dot2_f32_f16); the
 * reconstruction, the BLAS-1 updates and every reduction are FP32 (scalars
 * FP64).  BF16 storage: FP32 arithmetic throughout.  BF16 (8 exponent bits,
 * 7 fraction bits) is the alternative inner format the paper's conclusion
 * proposes to compare. */
typedef enum { QCD_FP64 = 0, QCD_FP32 = 1, QCD_FP16 = 2, QCD_BF16 = 3 } qcd_prec;
/* Flag for qcd_gauge_upload's prec_mask: store all 18 reals of every link
 * even when the field is in SU(3). */
enum { QCD_LINKS_FULL = 1 << 8 };
typedef enum { QCD_LAYOUT_CANONICAL = 0, QCD_LAYOUT_NATIVE = 1 } qcd_layout;
/* D = 1 - kappa H (eq. (1)); H is the hopping sum; D^dag = gamma_5 D gamma_5. */
/* QCD_OP_SCHUR: the even-odd matrix of eq. (5), out_e = in_e - kappa^2 H_eo H_oe in_e on even sites,
 * out_o = 0 (in_o is not read). */
typedef enum { QCD_OP_D = 0, QCD_OP_H = 1, QCD_OP_DDAG = 2, QCD_OP_HDAG = 3, QCD_OP_SCHUR = 4 } qcd_op;

typedef struct qcd_gauge qcd_gauge; /* opaque handle */
typedef struct qcd_ptc qcd_ptc;     /* opaque handle of the learned preconditioner (declared below) */

/* Parameters of the rescaled BiCGStab (Alg. 4; Alg. 5 when sigma_lambda > 0). */
typedef struct {
  double tol;          /* stop when |r| / gamma' <= tol * |b| (relative, unscaled residual) */
  int max_iter;        /* iteration cap (> 0) */
  double sigma;        /* rescale the residual to norm sigma after each iteration; 0 = off (gamma = 1) */
  double sigma_lambda; /* rescale the solution to norm sigma_lambda (Alg. 5); 0 = off */
  int recalc_gamma;    /* 1: gamma is the measured ratio |r stored| / |r before rescaling| */
  double omega0;       /* omega prescription threshold; the paper uses 0.7; 0 disables */
  int ftz;             /* 1: a binary16 store below 2^-14 (BF16: 2^-126) in magnitude is flushed to zero */
  int check_every;     /* > 0: host polls the convergence flag every this many iterations (and, in
                          qcd_solve_mixed_ir, drives each refinement step itself); 0: adaptive (qcd_bicgstab:
                          first poll after 4, then after the number the convergence rate predicts;
                          qcd_solve_mixed_ir: the steps run from the device, see there) */
  int use_graph;       /* 1: one iteration is captured in a hip graph (on a stream the handle owns) and
                          replayed; results are identical to plain launches */
  int even_odd;        /* 1: solve the even-odd preconditioned system of eq. (4)-(6) (the paper's form):
                          (1 - kappa^2 H_eo H_oe) x_e = b_e + kappa H_eo b_o on even sites, then
                          x_o = b_o + kappa H_oe x_e; vectors of the iteration are half-size.  In
                          qcd_solve_mixed_ir (through its inner parameters) the refinement runs on the
                          even system too, with its stop test taken relative to the full |b|; the
                          reported residual is always the full |b - D x| / |b|.  tol in qcd_bicgstab
                          is relative to |b_e + kappa H_eo b_o|. */
} qcd_bicgstab_params;

/* Parameters of the rescaled iterative refinement (Alg. 3; Alg. 2 is s = 1, recalc_shat = 0). */
typedef struct {
  double tol;               /* stop when |b - D x|_2 / |b|_2 <= tol, checked in FP64 */
  int max_outer;            /* outer iteration cap (> 0) */
  qcd_prec inner_prec;      /* storage precision of the inner solve (FP16, BF16, FP32 or FP64) */
  double s;                 /* the residual is rescaled to norm s before conversion */
  int recalc_shat;          /* 1: correct with s^ = |single(y~)| (Alg. 3); 0: with s */
  qcd_bicgstab_params inner;/* inner.tol is eps_tol (the paper's eps_tol^2 = 1e-4 is tol = 1e-2) */
  const qcd_ptc* precond;   /* NULL, or a network (built on the same gauge handle; it takes the right-hand
                               sides max_batch at a time) used as right preconditioner M of the FP16 inner
                               solve: the inner BiCGStab solves
                               (D c M) u = y~ and the refinement step corrects with t = c M u.  A step whose
                               FP64 residual does not drop, or that goes non-finite, is undone and the call
                               continues without the network (flexible refinement: the outer FP64 residual
                               is recomputed every step, so M may differ from D^-1 by any amount).  With
                               inner.even_odd the even system is preconditioned by the even-even block of M:
                               z = even rows of c M (v, 0), since the even-even block of D^-1 is the inverse
                               of the matrix of eq. (5) */
  double precond_scale;     /* c above; 0 = 1 / (largest |M v| / |v| over the first inner right-hand sides),
                               which keeps the FP16 vectors in the range of the plain solver */
} qcd_ir_params;

typedef struct {
  int outer_iters;          /* refinement steps (0 for qcd_bicgstab) */
  int inner_iters;          /* BiCGStab iterations in total */
  int matvec_low;           /* applications of D in the inner precision */
  int matvec_fp64;          /* FP64 applications of D (outer residuals, final check) */
  double true_rel_residual; /* |b - D x| / |b| in FP64 at return */
  double seconds;           /* wall-clock time inside the call */
  int inner_status;         /* last inner-solver stop reason: 1 converged, 2 max_iter, 3 non-finite, 4 breakdown */
  double first_shat_over_s; /* s^/s of the first refinement step (rounding of the FP16 conversion) */
  double* history;          /* optional caller-owned host array: (|r|/gamma')^2/|b|^2 per inner iteration,
                               concatenated over refinement steps */
  int history_cap;          /* capacity of history */
  int history_len;          /* entries written */
  double* outer_history;    /* optional caller-owned host array: |r|/|b| after each refinement step */
  int outer_history_cap;
  double* zeros;            /* optional: zero reals in y~ per refinement step (Fig. 9 diagnostic),
                               capacity outer_history_cap */
  int precond_steps;        /* refinement steps of the call whose inner solve used the network (the same
                               for every right-hand side of the call) */
  int precond_fallback;     /* refinement step at which the network was dropped, or -1 */
  double precond_scale;     /* the scale c used (0 without a network) */
} qcd_solve_info;

/* Message for the last error on this thread ("" if none). */
const char* qcd_last_error(void);

/* Gauge upload.  Converts the canonical FP64 field U_dev (complex128
 * [V][4][3][3], device) to native copies in the precisions selected by
 * prec_mask (bit (1 << QCD_FP64) etc.; 0 selects all four; the FP64 copy
 * is always built because the outer refinement needs it).  The handle owns
 * those copies and a reusable workspace; free it with qcd_gauge_free.
 * FP64 -> FP32/FP16/BF16 rounding is one round-to-nearest-even step.
 * Implements the low-precision matrix A~ of Alg. 3 (links stored in the
 * inner precision).  Synchronises with stream.  Errors: QCD_ERR_ARG for a
 * null pointer or an odd / < 2 extent, QCD_ERR_HIP on allocation failure. */
qcd_status qcd_gauge_upload(qcd_gauge** g, const int dims[4], const void* U_dev, int prec_mask, void* stream);
qcd_status qcd_gauge_free(qcd_gauge* g);
/* Reals stored per link in precision prec: 12 when every link passed the
 * SU(3) check at upload (row 2 equals conj(row0 x row1) to within 1e-14,
 * 1e-7, 1e-4, 1e-3 for FP64, FP32, FP16, BF16; the kernels rebuild row 2, which saves a
 * third of the link bytes), 18 otherwise or with QCD_LINKS_FULL; 0 if the
 * handle holds no links in prec. */
int qcd_gauge_link_reals(const qcd_gauge* g, qcd_prec prec);

/* Launch shape of the Wilson operator for precision prec (picked by a tuner):
 * sched 0 orders thread blocks by half-lattice index; sched m = 1..3 gives
 * each of the GPU's eight XCDs its own slab of z, swept in t order as 2^(m-1)
 * thinner sub-slabs one after the other (applies when (Lx/2)*Ly is a multiple
 * of the block's half-sites and Lz of 8*2^(m-1), else falls back to 0);
 * sched 4 gives each XCD a slab of t, swept in z order (applies when
 * (Lx/2)*Ly is a multiple of the block's half-sites and Lt of 8);
 * variant 0..5 selects how many hops' loads are prefetched while one hop is
 * computed and the minimum waves per SIMD the kernel is compiled for:
 * 0 (1 hop, 2 waves), 1 (2, 2), 2 (0, 3), 3 (1, 3), 4 (0, 4), 5 (1, 4), and 6:
 * the x and y neighbour spinors staged once per block in LDS, in the plain
 * operator on full fields (FP16 and BF16, when blocks of 128 half sites per
 * parity cover whole x rows) and in the one-parity launches of the even-odd
 * solvers (every precision, when blocks of 256 half sites cover whole x rows;
 * x extent at most 128, 64 for FP64), one right-hand side per launch tile;
 * otherwise as 1; 7: the same LDS forms with two hops prefetched in 16-bit
 * storage (one in FP32 and FP64), otherwise as 0.
 * rhs_tile (0 = automatic, 1, 2, 4) is the number of right-hand sides whose
 * lanes share one wave's link loads in a multi-RHS application, -2, -3, -4 the
 * number a thread applies one loaded link to (it must divide nrhs, else 1 is
 * used; automatic takes 3 or 2 per thread for FP16 and 1 otherwise); 8 selects
 * the matrix-core form for FP16 storage: the SU(3) products of a hop for a
 * tile of 16, 12, 8, 6 or 4 right-hand sides (the largest dividing nrhs) run
 * as binary16 16 x 16 x 16 matrix-core products, two sites per instruction;
 * it applies to the plain operator (launches with a reduction epilogue and
 * other precisions use one right-hand side per thread).  Results do not
 * depend on these choices beyond FP16 rounding of the tiles' summation order. */
qcd_status qcd_set_dslash_tuning(qcd_gauge* g, qcd_prec prec, int sched, int variant, int rhs_tile);
qcd_status qcd_get_dslash_tuning(const qcd_gauge* g, qcd_prec prec, int* sched, int* variant, int* rhs_tile);

/* Autotuner for the Wilson operator: times every launch choice (schedule,
 * variant, rhs_tile) for (prec, nrhs) with HIP events over reps launches on
 * scratch fields (allocated and freed here) and sets the fastest on the
 * handle; best_us (may be NULL) receives its time.  With cache_path (may be
 * NULL), a JSON-lines file keyed by lattice, precision, nrhs and GPU
 * architecture is read first and the result appended.  Synchronises. */
qcd_status qcd_autotune_dslash(qcd_gauge* g, qcd_prec prec, int nrhs, int reps, const char* cache_path,
                               double* best_us, void* stream);

/* Bytes of one native spinor field in precision prec. */
size_t qcd_spinor_bytes(const qcd_gauge* g, qcd_prec prec);

/* Workspace bytes that qcd_solve_mixed_ir (what = 0; what = 3 with a network
 * preconditioner), qcd_bicgstab (what = 1) or qcd_dslash with canonical
 * layout (what = 2) need, what = 0, 1 or 3 plus 8 for the even-odd form, for inner precision
 * prec, max_iter history entries and nrhs right-hand sides.  The size depends
 * on the handle's current launch tuning (the operator's partial-sum rows per
 * right-hand side): query it again after qcd_set_dslash_tuning or
 * qcd_autotune_dslash.  max_iter must be the inner iteration cap the call
 * uses.  Passing ws = NULL to those calls makes the handle's own cached
 * workspace be used (allocated on first use, grown when a call needs more;
 * a handle is not safe for concurrent calls). */
size_t qcd_workspace_bytes(const qcd_gauge* g, int what, qcd_prec prec, int max_iter, int nrhs);

/* Synthetic sources on the device (the right-hand sides of the training pairs
 * of the learned preconditioner, generated where they are used): ncomplex
 * complex128 values z = (g0 + i g1) / sqrt(2), E|z|^2 = 1, written to out_dev
 * in order.  Value j is the Box-Muller pair of draws 2j and 2j + 1 of a
 * counter-based SplitMix64 stream keyed by seed (Steele, Lea and Flood 2014),
 * so the values depend only on (seed, j).  Asynchronous on stream.  Errors:
 * QCD_ERR_ARG for a null pointer or ncomplex < 0. */
qcd_status qcd_gaussian_spinors(void* out_dev, int64_t ncomplex, uint64_t seed, void* stream);

/* Precision conversion with rescaling (Alg. 3, the steps y = alpha r and
 * y~ = low_prec(y)): native_dev = round_prec(scale * canonical_dev) with
 * one round-to-nearest-even conversion from FP64, optional flush to
 * zero of binary16 subnormals; if norm2 is not NULL it receives
 * sum |stored|^2 computed per site in the arithmetic precision and in FP64
 * across sites (the s^ of Alg. 3 is its square root).  Synchronises when
 * norm2 is requested. */
qcd_status qcd_convert(const qcd_gauge* g, qcd_prec prec, int nrhs, void* native_dev, const void* canonical_dev,
                       double scale, int ftz, double* norm2, void* stream);

/* Inverse conversion: canonical_dev (complex128) = scale * double(native_dev). */
qcd_status qcd_unconvert(const qcd_gauge* g, qcd_prec prec, int nrhs, void* canonical_dev, const void* native_dev,
                         double scale, void* stream);

/* Wilson operator (eq. (1), Alg. 1 with the projection of Sec. 2):
 * out = op(in) with op one of D, H, D^dag, H^dag.  prec selects the link
 * copy, the storage of in/out (native layout) and the arithmetic (FP64 for
 * FP64; FP32 for FP32 and BF16; for FP16 the binary16 projection and exact
 * binary16 link products summed in FP32 described at qcd_prec, FP32
 * reconstruction).  With QCD_LAYOUT_CANONICAL, in and out are
 * complex128 canonical fields, converted to/from prec around the
 * application.  With nrhs > 1 the links are read once per site for all
 * right-hand sides (a wave's lanes interleave sites and right-hand sides).
 * out must not alias in.  Asynchronous on stream. */
qcd_status qcd_dslash(const qcd_gauge* g, double kappa, qcd_op op, qcd_prec prec, qcd_layout layout, int nrhs,
                      void* out_dev, const void* in_dev, void* stream);

/* FP64 true residual of Alg. 3: r = b - D x (canonical complex128), and if
 * norm2 is not NULL, |r|^2.  Synchronises when norm2 is requested. */
qcd_status qcd_residual(const qcd_gauge* g, double kappa, int nrhs, void* r_dev, const void* x_dev, const void* b_dev,
                        double* norm2, void* stream);

/* Rescaled BiCGStab (Alg. 4 / Alg. 5) solving D x = b in precision prec,
 * x0 = 0, r* = b.  b_dev and x_dev are canonical complex128; b is rounded to
 * prec, the solution is returned in FP64 as x = lambda-unscaled inner x.
 * info (may be NULL) receives counts and the FP64 true residual.
 * Returns QCD_OK, QCD_NOT_CONVERGED, QCD_ERR_NONFINITE or QCD_ERR_BREAKDOWN
 * (x holds the last iterate in the last three cases).  Synchronises. */
qcd_status qcd_bicgstab(const qcd_gauge* g, double kappa, qcd_prec prec, int nrhs, void* x_dev, const void* b_dev,
                        const qcd_bicgstab_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* FP64 iterative refinement around the rescaled low-precision BiCGStab
 * (Alg. 3 with Alg. 4 / Alg. 5; Alg. 2 when s = 1 and recalc_shat = 0):
 *   x = 0, r = b; while |r|/|b| > tol: y~ = low(r s/|r|), s^ = |single(y~)|,
 *   solve A~ t = y~, x += (|r|/s^) double(t), r = b - D x (FP64).
 * b_dev, x_dev canonical complex128.  nrhs right-hand sides are solved
 * together: every kernel handles all of them, each with its own scalars,
 * and a right-hand side that has met the tolerance is skipped by the kernels
 * (per-right-hand-side masks).  With p->inner.check_every = 0, no network or
 * inner history and max_outer <= 128, the refinement steps run from the
 * device: the host
 * queues blocks of inner iterations, each followed by the kernels of one
 * refinement step that act only for right-hand sides whose inner solve has
 * stopped, and polls after as many blocks as the convergence so far predicts
 * (the first poll's block sizes come from the handle's previous such call
 * with the same tolerances); results are bit for bit those of host-driven
 * steps (check_every > 0).  Returns (the worst over right-hand sides)
 * QCD_OK when the FP64 true residual reaches tol, QCD_NOT_CONVERGED after
 * max_outer steps (x valid), QCD_ERR_NONFINITE / QCD_ERR_BREAKDOWN if an
 * inner solve failed before any progress.  Synchronises. */
qcd_status qcd_solve_mixed_ir(const qcd_gauge* g, double kappa, int nrhs, void* x_dev, const void* b_dev,
                              const qcd_ir_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * refinement of qcd_solve_mixed_ir (same arguments and results, bit for bit
 * the same kernels) with its workspace in a fixed 64 MiB device array of the
 * library instead of a caller or handle buffer.  The array exists once per
 * GPU from module load to process end; its address is looked up at
 * qcd_gauge_upload.  This call allocates nothing and creates no HIP object.
 * Limits: the workspace qcd_workspace_bytes() reports for the call (what = 0,
 * | 8 with inner.even_odd) must fit in 64 MiB, else QCD_ERR_WORKSPACE before
 * any launch (16^4 with one right-hand side fits); p->precond must be NULL and
 * p->inner.use_graph 0 (QCD_ERR_UNSUPPORTED).  Every call on a GPU shares that
 * GPU's array, which keeps the last call's contents (nothing in it needs to
 * start at zero): calls that overlap on one GPU (several host threads, or
 * streams that run concurrently) race and corrupt each other.
 * Synchronises. */
qcd_status qcd_solve_mixed_ir_static(const qcd_gauge* g, double kappa, int nrhs, void* x_dev, const void* b_dev,
                                     const qcd_ir_params* p, qcd_solve_info* info, void* stream);

/* Several lattices in one call (the batched form of Alg. 3): nlat gauge
 * handles (distinct, possibly of different extents), each with its own kappa,
 * nrhs right-hand sides b_dev[i] and solutions x_dev[i] (canonical complex128,
 * device), solved with the same parameters p.  Every refinement step converts
 * all lattices, runs their inner BiCGStab iterations together (each lattice
 * on its handle's own stream, forked from and joined to `stream`, so small
 * lattices run concurrently; with p->inner.use_graph each lattice replays its
 * captured iteration) and corrects them; the host polls all lattices' device
 * scalars with one synchronisation.  Per right-hand side results match
 * qcd_solve_mixed_ir on that lattice alone.  info may be NULL or hold nlat
 * arrays of nrhs[i] entries.  Workspaces: ws may be NULL (every lattice uses
 * its handle's cached workspace, allocated or grown as in qcd_solve_mixed_ir)
 * or hold nlat caller-owned device buffers, ws[i] of ws_bytes[i] >=
 * qcd_workspace_bytes(g[i], 0 (| 8 with inner.even_odd), inner_prec,
 * inner.max_iter, nrhs[i]) bytes (a NULL entry selects that handle's own);
 * with every ws[i] given the call allocates no device memory and creates no
 * HIP objects (the streams and events it forks onto were made at upload).
 * p->precond must be NULL (QCD_ERR_UNSUPPORTED otherwise: a network is bound
 * to one gauge handle; several right-hand sides of one lattice take it through
 * qcd_solve_mixed_ir).  nlat in 1..64.
 * QCD_ERR_WORKSPACE if a ws[i] is too small. */
qcd_status qcd_solve_mixed_ir_batched(int nlat, const qcd_gauge* const* g, const double* kappa, const int* nrhs,
                                      void* const* x_dev, const void* const* b_dev, const qcd_ir_params* p,
                                      qcd_solve_info* const* info, void* const* ws, const size_t* ws_bytes,
                                      void* stream);

/* Estimates of the largest and smallest |eigenvalue| of the even-odd matrix
 * A = 1 - kappa^2 H_eo H_oe of eq. (5), the ratio Sec. 6 quotes for its test
 * configuration (a diagnostic of the conditioning of the synthetic fields).
 * Largest: power_iters steps of x <- A x / |A x| in FP64 from the even half
 * of the Gaussian field with the given seed; abs_max is the geometric mean of
 * |A x_k| over the second half of the steps (a complex-conjugate pair at the
 * top, which gamma_5-hermiticity allows, makes single ratios oscillate; the
 * mean then converges as 1 / power_iters).  Smallest: the same with
 * x <- A^-1 x / |A^-1 x| for inverse_iters steps (seed + 1), where A^-1 x is
 * the even half of the solution of D y = (x on even sites, 0 on odd sites)
 * from qcd_solve_mixed_ir (even-odd, FP16 inner if the handle holds FP16
 * links, else FP64; tolerance 1e-12); abs_min = 1 / the mean, NaN if
 * inverse_iters = 0.  Needs FP64 links.  Allocates and frees its own buffers
 * (three one-parity FP64 fields and two canonical fields); synchronises.
 * Errors: QCD_ERR_ARG (null handle or output, kappa not positive, power_iters
 * outside 2..100000, inverse_iters outside 0..1000), QCD_NOT_CONVERGED if a solve stops short,
 * QCD_ERR_NONFINITE, QCD_ERR_HIP. */
qcd_status qcd_eo_spectrum(const qcd_gauge* g, double kappa, int power_iters, int inverse_iters, uint64_t seed,
                           double* abs_max, double* abs_min, void* stream);

/* Memory-system probe (a diagnostic; not part of the method): the average
 * time in microseconds of one sweep over bytes (a positive multiple of 16)
 * that reads src_dev (mode 0), copies src_dev to dst_dev (mode 1) or writes
 * dst_dev (mode 2), every lane moving 16-byte granules with non-temporal
 * loads and stores, timed with HIP events over reps (1..10000) sweeps after
 * one untimed sweep.  dst_dev holds bytes (mode 0 may store there only if
 * the data read happens to hash to a fixed pattern).  The bandwidth the
 * Wilson operator is compared with is measured this way on the same GPU.
 * Synchronises.  QCD_ERR_ARG for invalid arguments. */
qcd_status qcd_stream_probe(void* dst_dev, const void* src_dev, size_t bytes, int mode, int reps, double* us,
                            void* stream);

/* ------------------------------------------------------------------------
 * Learned preconditioner: a gauge-covariant parallel-transport network.
 * A layer maps C_in spinor fields to C_out fields,
 *   out_j(x) = sum_i sum_p W[p][j][i] (T_p psi_i)(x),
 * over nine paths p = 0, +x, -x, +y, -y, +z, -z, +t, -t (in that order) with
 *   (T_{+mu} psi)(x) = U_mu(x) psi(x + mu), (T_{-mu} psi)(x) = U_mu(x - mu)^dag psi(x - mu),
 * and W[p][j][i] a complex 4x4 spin matrix [s'][s].  Layers compose linearly
 * (a fixed linear, gauge-covariant operator M).  Channel mixing runs on BF16
 * matrix cores with FP32 accumulation; activations are FP32.  This is not a
 * construction of the paper; the solver uses M as a right preconditioner of
 * its inner BiCGStab (qcd_ir_params.precond).
 */

/* Create a network of nlayers layers with channels[0..nlayers] spinor fields
 * per layer boundary (channels[0] = channels[nlayers] = 1, others 1 or 2) on
 * the lattice of g (which must hold FP32 links; the handle keeps a pointer
 * to g, which must outlive it), for batches of up to max_batch fields.
 * Weights start at zero.  Device buffers are owned by the handle; those of
 * the two-pass form (training, the loss and gradient calls, FP32 mixing) are
 * allocated by the first call that uses it, so a handle that only
 * preconditions holds the activations of max_batch fields and no more. */
qcd_status qcd_ptc_create(qcd_ptc** net, const qcd_gauge* g, int nlayers, const int* channels, int max_batch,
                          void* stream);
qcd_status qcd_ptc_free(qcd_ptc* net);
/* Point the network at another gauge field with the same extents (training
 * over several fields with one set of weights and optimiser state). */
qcd_status qcd_ptc_set_gauge(qcd_ptc* net, const qcd_gauge* g);
/* Precision of the channel mixing in the two-pass form (training, the loss
 * and gradient calls, and qcd_ptc_apply): QCD_BF16 (the default; inputs,
 * weights and output gradients rounded to BF16 on the BF16 matrix cores) or
 * QCD_FP32 (all of them FP32 on the FP32 matrix cores, for gradients that
 * agree with an FP64 reference to FP32 rounding).  The FP16 form that the
 * inner solver applies keeps BF16 mixing.  Reallocates the handle's GEMM
 * operands (FP32 doubles them); synchronises.  QCD_ERR_ARG for another
 * precision. */
qcd_status qcd_ptc_set_mixing(qcd_ptc* net, qcd_prec prec, void* stream);
/* Set the weights of a (1, 2, 2, 1) network to the third-order Neumann
 * series of the Wilson matrix, M = sum_{k=0..3} (kappa H)^k, so that
 * D M = 1 - (kappa H)^4 (with D = 1 - kappa H, eq. (1)).  Layers: (psi,
 * kappa H psi) -> (c0 + c1, kappa H (c0 + c1)) -> c0 + kappa H c1.  A
 * starting point for training.  Synchronises. */
qcd_status qcd_ptc_init_neumann(qcd_ptc* net, double kappa, void* stream);
/* Complex weights in total: sum over layers of 9 * C_out * C_in * 16. */
size_t qcd_ptc_num_weights(const qcd_ptc* net);
/* Host complex128 weights, layers concatenated, each [9][C_out][C_in][4][4];
 * setting them resets the optimiser state.  Synchronise. */
qcd_status qcd_ptc_set_weights(qcd_ptc* net, const double* w_host, void* stream);
qcd_status qcd_ptc_get_weights(const qcd_ptc* net, double* w_host, void* stream);
/* out = M(in) for nbatch canonical complex128 fields (device). */
qcd_status qcd_ptc_apply(qcd_ptc* net, int nbatch, void* out_dev, const void* in_dev, void* stream);
/* As qcd_ptc_apply, with the activations stored in prec: QCD_FP32 is
 * qcd_ptc_apply; QCD_FP16 rounds the input to binary16 and runs the layers as
 * an FP16 inner solve with qcd_ir_params.precond applies them (FP16 links and
 * activations, FP32 sums, the weights rounded to BF16 as above).  QCD_ERR_ARG
 * for another precision or, with QCD_FP16, a gauge handle without FP16
 * links.  Inputs must lie within the binary16 range. */
qcd_status qcd_ptc_apply_prec(qcd_ptc* net, qcd_prec prec, int nbatch, void* out_dev, const void* in_dev,
                              void* stream);
/* Loss (1/B) sum_b |M(r_b) - e_b|^2 / |e_b|^2 and, if grad_host is not NULL,
 * its gradient dL/dRe W + i dL/dIm W (host complex128, layout of the
 * weights).  r_dev, e_dev: nbatch canonical complex128 fields.  Synchronises. */
qcd_status qcd_ptc_loss_grad(qcd_ptc* net, int nbatch, const void* r_dev, const void* e_dev, double* loss,
                             double* grad_host, void* stream);
/* The residual loss (1/B) sum_b |D M(r_b) - r_b|^2 / |r_b|^2, with D the
 * Wilson matrix of eq. (1) at kappa (FP32 operator on the handle's FP32
 * links), and if grad_host is not NULL its gradient in the layout of the
 * weights.  It measures how far D M is from the identity on the sources, the
 * quantity a right preconditioner is judged by, and needs no solves
 * (r_dev: nbatch canonical complex128 fields).  Synchronises.  QCD_ERR_ARG
 * for kappa not positive and finite. */
qcd_status qcd_ptc_loss_grad_residual(qcd_ptc* net, double kappa, int nbatch, const void* r_dev, double* loss,
                                      double* grad_host, void* stream);
/* One Adam step (as qcd_ptc_train_step) on the residual loss above. */
qcd_status qcd_ptc_train_step_residual(qcd_ptc* net, double kappa, int nbatch, const void* r_dev, double lr,
                                       double* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 weights with
 * learning rate lr; loss (may be NULL) receives the loss before the step. */
qcd_status qcd_ptc_train_step(qcd_ptc* net, int nbatch, const void* r_dev, const void* e_dev, double lr, double* loss,
                              void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QCD_H */
