// Declarations shared by the library's translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"
#include "qcd.h"

namespace qcd {

enum { kFP64 = 0, kFP32 = 1, kFP16 = 2, kBF16 = 3 };
constexpr int kNumPrec = 4;
enum { kOpD = 0, kOpH = 1, kOpDdag = 2, kOpHdag = 3 };
enum { kEpiNone = 0, kEpiDotAux = 1, kEpiTS = 2, kEpiResid = 3, kEpiTSAux = 4, kEpiRecon = 5 };
// kEpiRecon (FP64, one parity, D form with kappa < 0): out = cin - kappa H in is
// stored, and |cin - (out + kappa H in)|^2 goes to the partials: the residual
// rows of the stored out, from the same hop sum (the odd rows of b - D x when
// the even-odd solve rebuilds x_o).

// Inner-solver status codes kept on the device.
enum { kRunning = 0, kConverged = 1, kMaxIter = 2, kNonFinite = 3, kBreakdown = 4 };

constexpr int kMaxRhs = 64;  // right-hand sides per call
constexpr int kPtcMaxLayers = 4;  // layers of the parallel-transport network

// Record an error message for qcd_last_error(); returns code.
int set_error(int code, const char* fmt, ...);

inline size_t prec_complex_bytes(int prec) { return prec == kFP64 ? 16 : (prec == kFP32 ? 8 : 4); }  // FP16, BF16: 4

// Scalars of the rescaled BiCGStab (Alg. 4 / Alg. 5) and of the outer
// refinement (Alg. 2 / Alg. 3), all FP64, resident in device memory.
// Complex values are (re, im) pairs.
struct Scalars {
  // parameters
  double sigma;          // residual norm after rescaling (0: gamma = 1)
  double sigma_lambda;   // solution norm after rescaling (0: lambda = 1)
  double omega0;         // omega prescription threshold
  double tol2;           // inner stop: (|r|/gamma')^2 <= tol2 * |b|^2
  int recalc_gamma;
  int max_iter;
  // BiCGStab recurrences
  double bnorm2;
  double rho[2], rho_prev[2];    // rho = (r*, r), rho' (rescaled)
  double alpha[2], alpha_prev[2];
  double omega[2], omega_prev[2];
  double beta[2];
  double pcoef[2];               // beta * gamma: folds the p, v rescaling into the next p update
  double xcoef;                  // lambda' / gamma' for the x update
  double xscale;                 // pending lambda, applied to x at the next x update
  double gamma_pred;             // factor applied to the new residual when stored
  double gamma, gamma_cum, lambda_cum;
  double rnorm2;                 // |r_stored|^2
  int iter;
  int first;                     // first iteration: p = r, x = 0
  int active;                    // 0 once the solver stopped
  int status;
  int outer_active;              // 0 once this right-hand side met the outer tolerance
  // outer refinement
  double out_rnorm;              // |r| of the FP64 residual
  double out_scale;              // s / |r|
  double shat;                   // |single(y~)|
  double zeros;                  // zero reals in y~
  double out_bnorm;              // |b|, for the outer stopping test
  double out_tol;
  // device-driven refinement: the stop of an inner solve raises outer_step, and
  // the refinement step's kernels (correction, FP64 residual, its norm, the
  // conversion and the next inner start) act only on right-hand sides that
  // have it, so a captured graph of iterations and one step runs several
  // refinement steps between host polls
  int dev_outer;                 // 1: device-driven refinement for this right-hand side
  int outer_step;                // 1 from the stop of an inner solve until its refinement step is done
  int outer_count;               // refinement steps done (device-driven)
  int inner_total;               // inner iterations over all steps (device-driven)
  int max_outer;                 // refinement step cap (device-driven)
  int fail;                      // status of the inner solve that ended refining (kNonFinite, kBreakdown), else 0
  int last_status;               // stop reason of the last inner solve (device-driven)
  int pad_i;
  double first_shat;             // s^ of the first refinement step (device-driven)
  double bfull;                  // |b| of the full system (device-driven start)
};
// refinement steps whose |r| and zero count the device-driven refinement logs per right-hand side
constexpr int kOuterLog = 128;

// Launch choices of the Wilson operator (picked by the tuner).
struct DslashTune {
  int sched;    // 0: blocks in half-index order; m = 1..3: XCD z slabs (each swept as 2^(m-1) sub-slabs);
                // 4: XCD t slabs swept in z order
  int variant;  // (hops prefetched, min waves per SIMD): 0 (1,2), 1 (2,2), 2 (0,3), 3 (1,3), 4 (0,4), 5 (1,4)
                // (prefetching 2 hops at 5 waves spills registers and measured slower in every precision);
                // 6: x and y neighbours staged in LDS (the FP16 / BF16 plain full-lattice operator and the
                // one-parity launches of every precision, one right-hand side; else as 1); 7: as 6 with two
                // hops prefetched in 16-bit storage, else as 0
  int rhs_tile; // right-hand sides sharing a link: 0 = automatic; 1, 2, 4 = that many in adjacent lanes;
                // -2, -3, -4 = that many per thread (link loaded and rebuilt once in registers);
                // 8 = the matrix-core form (kRhsTileMfma)
  int recon;    // links stored as 6 entries (rows 0, 1; row 2 rebuilt) instead of 9: a property of the data
};
constexpr int kDslashVariants = 8;
// rhs_tile code of the matrix-core form (FP16 storage, plain operator; 4, 6, 8, 12 or 16 right-hand sides per tile)
constexpr int kRhsTileMfma = 8;
// right-hand sides per matrix-core tile for n right-hand sides (0: the form does not apply)
inline int mfma_rhs_tile(int n) {
  const int cand[5] = {16, 12, 8, 6, 4};
  for (int i = 0; i < 5; i++)
    if (n % cand[i] == 0) return cand[i];
  return 0;
}
struct DslashSched {
  int mode, nsb, ntiles, Lz, Lt, bp, zc, sub, H;  // H: half-sites per parity per block
};
constexpr int kDslashScheds = 5;
DslashSched make_sched(const Geom& g, int mode, int T, int n, bool eo = false);
int rhs_tile_for(const DslashTune& tune, int n);
// right-hand sides per thread (rhs_tile = -R, R = 2..4, n divisible by R), else 1
int reg_tile_for(const DslashTune& tune, int n);

// Every launcher takes n, the number of right-hand sides: vector arguments
// hold n native spinors back to back (stride spinor_elems), sc points to
// Scalars[n], and partial sums are laid out [rhs][row][value].

// launchers (dslash.hip)
// mask (with scal): 0 computes the right-hand sides whose inner solve is active, 1 those whose
// device-driven refinement step is due (outer_step)
void launch_dslash(int prec, const Geom& g, const DslashTune& tune, int op, int epi, int n, void* out, const void* in,
                   const void* U, double kappa, const void* aux, double* partials, const Scalars* scal, int ftz,
                   hipStream_t st, const void* cin = nullptr, int eo_par = -1, int mask = 0);
int dslash_partial_rows(const Geom& g, const DslashTune& tune, int n, bool eo = false);  // rows per right-hand side

// launchers (blas.hip)
int site_grid(const Geom& g);              // blocks (and partial rows) per right-hand side, site-ordered kernels
int flat_rows(const Geom& g, int prec);    // blocks (and partial rows) per right-hand side, BLAS-1 kernels
void launch_pack_links(const Geom& g, int prec, void* dst, const double* Ucanon, int recon, hipStream_t st);
// out = largest deviation of a link's row 2 from conj(row0 x row1); partials: site_grid(g) doubles
void launch_link_su3_dev(const Geom& g, const double* Ucanon, double* partials, double* out, hipStream_t st);
void launch_pack_spinor(const Geom& g, int prec, int n, void* dst, const double* canon, double scale, int ftz,
                        double* partials, hipStream_t st);
void launch_unpack_spinor(const Geom& g, int prec, int n, double* canon, const void* src, const double* scale_dev,
                          double scale, hipStream_t st);
// FP64 only: canonical <-> two one-parity native fields (even sites in `even`,
// odd sites in `odd`, each with a one-parity field per right-hand side)
void launch_pack_spinor_split(const Geom& g, int n, void* even, void* odd, const double* canon, double* partials,
                              hipStream_t st);
void launch_unpack_spinor_split(const Geom& g, int n, double* canon, const void* even, const void* odd,
                                hipStream_t st);
void launch_zero(const Geom& g, int prec, int n, void* dst, hipStream_t st);
// n one-parity fields (geometry gh) copied; right-hand side b of dst / src starts
// b * dst_stride / b * src_stride stored complex numbers in
void launch_copy_fields(const Geom& gh, int prec, int n, void* dst, size_t dst_stride, const void* src,
                        size_t src_stride, hipStream_t st);
// ncomplex complex normal values (canonical complex128) from a counter-based stream keyed by seed
void launch_gaussian(double* out, int64_t ncomplex, uint64_t seed, hipStream_t st);
// native FP64 -> native prec (RNE, |stored|^2 partials if not null); native prec -> FP64 times scale_dev[rhs]
void launch_narrow(const Geom& g, int prec, int n, void* dst, const double* src, double* partials, int ftz,
                   hipStream_t st);
void launch_widen(const Geom& g, int prec, int n, double* dst, const void* src, const double* scale_dev,
                  hipStream_t st);

void launch_bicg_init(int n, Scalars* sc, const double* partials, int nrows, hipStream_t st);
void launch_p_update(const Geom& g, int prec, int n, Scalars* sc, void* p, const void* v, const void* r, int ftz,
                     hipStream_t st);
void launch_alpha(int n, Scalars* sc, const double* partials, int nrows, hipStream_t st);
void launch_s_update(const Geom& g, int prec, int n, Scalars* sc, void* r, const void* v, int ftz, hipStream_t st);
void launch_omega(int n, Scalars* sc, const double* partials, int nrows, hipStream_t st);
void launch_xr_update(const Geom& g, int prec, int n, Scalars* sc, void* x, void* r, const void* t, const void* p,
                      const void* rstar, double* partials, int ftz, hipStream_t st);
void launch_iter_end(int n, Scalars* sc, const double* partials, int nrows, double* history, int hist_stride,
                     hipStream_t st);

// x_o = eta_o + kappa t (t = H_oe x_e, one-parity FP64 fields) and the canonical solution
// from x_e and x_o in one pass (g: the full lattice); |odd residual rows|^2 partials,
// site_grid(half_geom(g)) rows per right-hand side
void launch_eo_recon_unpack(const Geom& g, int n, double* canon, const double* xe, const double* eta_o,
                            const double* t, double kappa, double* partials, hipStream_t st);
// start of the device-driven refinement: |b| (from b2_dev, or the start norm),
// the even-odd tolerance relative to it, and the step bookkeeping
void launch_ir_dev_start(int n, Scalars* sc, const double* b2_dev, double tol, int max_outer, hipStream_t st);
// with log (device-driven refinement): log[rhs][k] = (|r|, zeros of y~) of step k
void launch_outer_residual_norm(int n, Scalars* sc, const double* partials, int nrows, double s_target,
                                hipStream_t st, double* log = nullptr);
void launch_convert(const Geom& g, int prec, int n, Scalars* sc, const double* r64, void* y, void* rstar,
                    double* partials, int ftz, hipStream_t st);
void launch_convert_finish(int n, Scalars* sc, const double* partials, int nrows, int recalc_shat, double s_target,
                           hipStream_t st);
void launch_correct(const Geom& g, int prec, int n, Scalars* sc, double* x64, const void* xlo, hipStream_t st);
void launch_finish_sum(int n, const double* partials, int nrows, int nv, double* out, hipStream_t st);
// memory-system probe: mode 0 reads src, 1 copies src to dst, 2 writes dst (bytes a multiple of 16)
void launch_stream_probe(int mode, void* dst, const void* src, size_t bytes, hipStream_t st);

}  // namespace qcd

struct qcd_ptc;
struct qcd_gauge;
namespace qcd {
// network applied to nb native FP16 fields: out = scale * M(in), skipping
// batches whose solver stopped when scal is given (ptc.hip)
void ptc_apply_half(qcd_ptc* n, int nb, const void* in, void* out, float scale, int ftz, const Scalars* scal,
                    hipStream_t st);
// largest |M(v)| / |v| over nb native FP16 fields (synchronises)
qcd_status ptc_gain(qcd_ptc* n, int nb, const void* in, double* gain, hipStream_t st);
int ptc_max_batch(const qcd_ptc* n);
const qcd_gauge* ptc_gauge(const qcd_ptc* n);
}  // namespace qcd

// The gauge handle behind the C ABI's opaque qcd_gauge.
struct qcd_gauge {
  qcd::Geom g;
  int dims[4];
  void* U[qcd::kNumPrec];  // native links per precision (FP64, FP32, FP16, BF16)
  void* ws;          // cached workspace used when the caller passes none
  size_t ws_bytes;
  qcd::Scalars* host_sc;  // pinned mirror of the device scalars (kMaxRhs entries)
  double* host_log;       // pinned copy of the device-driven refinement's step log (kMaxRhs x kOuterLog x 2)
  qcd::DslashTune tune[qcd::kNumPrec];
  // one captured BiCGStab iteration, reused while its key (every value and
  // device address the captured launches bake in) is unchanged
  hipStream_t cap_stream;   // created at upload: capture, and this lattice's share of a batched solve
  hipEvent_t ev_fork, ev_done;  // created at upload: fork / join of a batched solve's streams
  hipGraphExec_t graph_exec;
  unsigned long long graph_key[32];
  double su3_dev;  // largest |row2 - conj(row0 x row1)| of the uploaded links (INFINITY if not checked)
  // what the last device-driven refinement on this handle took (inner iterations
  // per step, steps), with the parameters it ran with; a scheduling hint only
  int hint_iters, hint_steps;
  double hint_key[4];
};

