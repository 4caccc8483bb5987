// C-ABI of libqcd: gauge upload, Wilson operator, rescaled BiCGStab and the
// FP64 iterative refinement driver.  The host only sequences kernels and
// polls a small status record; every vector operation runs in the kernels of
// dslash.hip and blas.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qcd.h"
#include "internal.h"

using namespace qcd;

// struct qcd_gauge is defined in internal.h (shared with the network code).

static thread_local std::string g_err;

// Record an error message for qcd_last_error() and return code.
int qcd::set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace {

template <typename... A> qcd_status fail(qcd_status code, const char* fmt, A... a) {
  return (qcd_status)qcd::set_error((int)code, fmt, a...);
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(QCD_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define HIP_LAUNCHED()                                                                          \
  do {                                                                                          \
    hipError_t e_ = hipGetLastError();                                                          \
    if (e_ != hipSuccess) return fail(QCD_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// address of the static workspace on the current device (defined with it below)
qcd_status scratch_address(void** out);

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t spinor_bytes(const Geom& g, int prec) { return spinor_elems(g) * prec_complex_bytes(prec); }
size_t canon_bytes(const Geom& g) { return (size_t)2 * g.Vh * 12 * 16; }
int max_rows(const Geom& g, const DslashTune* tune, int n) {
  int rows = site_grid(g);
  for (int p = 0; p < kNumPrec; p++) rows = std::max(rows, flat_rows(g, p));
  for (int p = 0; p < kNumPrec; p++) rows = std::max(rows, dslash_partial_rows(g, tune[p], n));
  return rows;
}

// Workspace carve-up.
struct Carve {
  char* base;
  size_t off = 0;
  void* take(size_t b) {
    void* p = base ? base + off : nullptr;
    off += align256(b);
    return p;
  }
};

struct Work {
  int n = 1;
  double2* x64 = nullptr;
  double2* b64 = nullptr;
  double2* r64 = nullptr;
  void* x = nullptr;
  void* r = nullptr;
  void* rstar = nullptr;
  void* p = nullptr;
  void* v = nullptr;
  void* t = nullptr;
  void* z = nullptr;        // M p and M s of the preconditioned iteration
  double2* x64b = nullptr;  // x before a preconditioned refinement step
  // even-odd solve (eq. (4)-(6)): every vector is a one-parity field; inner
  // vectors, r64, x64 (= x_e) and eta_e are even, eta_o and x64o (= x_o) odd;
  // t1 / t64 hold H_oe of a vector
  bool eo = false;
  void* t1 = nullptr;
  double2 *eta_e = nullptr, *eta_o = nullptr, *bp64 = nullptr, *t64 = nullptr, *x64o = nullptr;
  // even-odd with a network: full FP16 fields around M (the odd halves of zin stay zero)
  void* zin = nullptr;
  void* zout = nullptr;
  double* partials = nullptr;
  Scalars* sc = nullptr;
  double* history = nullptr;
  int hist_stride = 1;
  double* sums = nullptr;
  double* scale = nullptr;
  double* outer_log = nullptr;  // device-driven refinement: (|r|, zeros) per step, kOuterLog steps per right-hand side
  size_t bytes = 0;
};

// what: 0 refinement, 1 BiCGStab, 2 operator with canonical layout, 3 preconditioned refinement;
// | kWhatEO: the even-odd form of 0, 1 or 3
constexpr int kWhatEO = 8;
Work carve(const qcd_gauge* G, int what_in, int prec, int max_iter, int n, char* base) {
  const Geom& g = G->g;
  const bool eo = (what_in & kWhatEO) != 0;
  const int what = what_in & 7;
  Carve c{base};
  Work w;
  w.n = n;
  if (eo && (what == 0 || what == 1 || what == 3)) {
    const Geom gh = half_geom(g);
    w.eo = true;
    w.eta_e = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.eta_o = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.bp64 = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.t64 = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.x64 = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.x64o = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.r64 = (double2*)c.take(n * spinor_bytes(gh, kFP64));
    w.x = c.take(n * spinor_bytes(gh, prec));
    w.r = c.take(n * spinor_bytes(gh, prec));
    w.rstar = c.take(n * spinor_bytes(gh, prec));
    w.p = c.take(n * spinor_bytes(gh, prec));
    w.v = c.take(n * spinor_bytes(gh, prec));
    w.t = c.take(n * spinor_bytes(gh, prec));
    w.t1 = c.take(n * spinor_bytes(gh, prec));
    w.hist_stride = max_iter > 0 ? max_iter : 1;
    w.history = (double*)c.take(sizeof(double) * (size_t)w.hist_stride * n);
    if (what == 3) {
      w.z = c.take(n * spinor_bytes(gh, prec));
      w.x64b = (double2*)c.take(n * spinor_bytes(gh, kFP64));
      w.zin = c.take(n * spinor_bytes(g, prec));
      w.zout = c.take(n * spinor_bytes(g, prec));
    }
  } else if (what == 0 || what == 1 || what == 3) {
    w.x64 = (double2*)c.take(n * spinor_bytes(g, kFP64));
    w.b64 = (double2*)c.take(n * spinor_bytes(g, kFP64));
    w.r64 = (double2*)c.take(n * spinor_bytes(g, kFP64));
    w.x = c.take(n * spinor_bytes(g, prec));
    w.r = c.take(n * spinor_bytes(g, prec));
    w.rstar = c.take(n * spinor_bytes(g, prec));
    w.p = c.take(n * spinor_bytes(g, prec));
    w.v = c.take(n * spinor_bytes(g, prec));
    w.t = c.take(n * spinor_bytes(g, prec));
    w.hist_stride = max_iter > 0 ? max_iter : 1;
    w.history = (double*)c.take(sizeof(double) * (size_t)w.hist_stride * n);
    if (what == 3) {
      w.z = c.take(n * spinor_bytes(g, prec));
      w.x64b = (double2*)c.take(n * spinor_bytes(g, kFP64));
    }
  } else {
    w.x = c.take(n * spinor_bytes(g, prec));
    w.r = c.take(n * spinor_bytes(g, prec));
  }
  w.partials = (double*)c.take((size_t)max_rows(g, G->tune, n) * 8 * sizeof(double) * n);
  w.sc = (Scalars*)c.take(sizeof(Scalars) * n);
  w.sums = (double*)c.take(8 * sizeof(double) * n);
  w.scale = (double*)c.take(sizeof(double) * n);
  if (what == 0 || what == 3) w.outer_log = (double*)c.take(sizeof(double) * 2 * kOuterLog * n);
  w.bytes = c.off;
  return w;
}

qcd_status get_work(const qcd_gauge* gc, int what, int prec, int max_iter, int n, void* ws, size_t ws_bytes,
                    Work* out) {
  qcd_gauge* g = const_cast<qcd_gauge*>(gc);
  Work need = carve(g, what, prec, max_iter, n, nullptr);
  char* base;
  if (ws) {
    if (ws_bytes < need.bytes)
      return fail(QCD_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need.bytes);
    base = (char*)ws;
  } else {
    if (g->ws_bytes < need.bytes) {
      if (g->ws) HIP_TRY(hipFree(g->ws));
      g->ws = nullptr;
      g->ws_bytes = 0;
      HIP_TRY(hipMalloc(&g->ws, need.bytes));
      g->ws_bytes = need.bytes;
    }
    base = (char*)g->ws;
  }
  *out = carve(g, what, prec, max_iter, n, base);
  return QCD_OK;
}

bool valid_prec(int p) { return p == kFP64 || p == kFP32 || p == kFP16 || p == kBF16; }

qcd_status check_gauge(const qcd_gauge* g, int prec) {
  if (!g) return fail(QCD_ERR_ARG, "null gauge handle");
  if (!valid_prec(prec)) return fail(QCD_ERR_ARG, "invalid precision %d", prec);
  if (!g->U[prec]) return fail(QCD_ERR_ARG, "gauge handle holds no links in precision %d", prec);
  return QCD_OK;
}

qcd_status check_nrhs(int n) {
  if (n < 1 || n > kMaxRhs) return fail(QCD_ERR_ARG, "nrhs must be in 1..%d", kMaxRhs);
  return QCD_OK;
}

// Canonical complex128 fields are read and written one complex (16 bytes) per access.
qcd_status check_canonical(const void* p, const char* what) {
  if (!p) return fail(QCD_ERR_ARG, "null %s", what);
  if ((uintptr_t)p & 15) return fail(QCD_ERR_ARG, "%s is not 16-byte aligned (complex128)", what);
  return QCD_OK;
}

qcd_status read_scalars(const qcd_gauge* g, const Work& w, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(g->host_sc, w.sc, sizeof(Scalars) * w.n, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return QCD_OK;
}

qcd_status read_sum(const Work& w, int nrows, int nv, double* out, hipStream_t st) {
  launch_finish_sum(w.n, w.partials, nrows, nv, w.sums, st);
  HIP_LAUNCHED();
  HIP_TRY(hipMemcpyAsync(out, w.sums, w.n * nv * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return QCD_OK;
}

void init_params(Scalars* h, const qcd_bicgstab_params& p) {
  memset(h, 0, sizeof(Scalars));
  h->sigma = p.sigma > 0 ? p.sigma : 0.0;
  h->sigma_lambda = p.sigma_lambda > 0 ? p.sigma_lambda : 0.0;
  h->omega0 = p.omega0;
  h->tol2 = p.tol * p.tol;
  h->recalc_gamma = p.recalc_gamma;
  h->max_iter = p.max_iter;
  h->outer_active = 1;
  h->out_bnorm = -1.0;
}

qcd_status check_bicg_params(const qcd_bicgstab_params* p) {
  if (!p) return fail(QCD_ERR_ARG, "null parameters");
  if (!(p->tol >= 0) || p->max_iter <= 0) return fail(QCD_ERR_ARG, "tol must be >= 0 and max_iter > 0");
  if (p->sigma < 0 || p->sigma_lambda < 0 || p->omega0 < 0 || p->omega0 > 1)
    return fail(QCD_ERR_ARG, "sigma, sigma_lambda >= 0 and 0 <= omega0 <= 1 required");
  return QCD_OK;
}

// The right preconditioner of the inner iteration: z = c M v (FP16 fields).
struct Precond {
  qcd_ptc* net = nullptr;
  float scale = 1.0f;
};

// z = c M v for n inner (FP16) vectors.  Even-odd: z = the even rows of c M (v, 0).
// The even-even block of D^-1 is the inverse of the Schur complement of
// eq. (5), so the even-even block of a network that approximates D^-1 is a
// right preconditioner of the even system (the third-order Neumann weights
// give 1 + kappa^2 H_eo H_oe there, the first-order series of its inverse).
void precond_apply(const qcd_gauge* g, const Precond& pc, const Work& w, int n, const void* v, void* z, int ftz,
                   const Scalars* sc, hipStream_t st) {
  if (!w.eo) {
    ptc_apply_half(pc.net, n, v, z, pc.scale, ftz, sc, st);
    return;
  }
  const Geom gh = half_geom(g->g);
  const size_t half = spinor_elems(gh), full = spinor_elems(g->g);
  launch_copy_fields(gh, kFP16, n, w.zin, full, v, half, st);
  ptc_apply_half(pc.net, n, w.zin, w.zout, pc.scale, ftz, sc, st);
  launch_copy_fields(gh, kFP16, n, z, half, w.zout, full, st);
}

// One BiCGStab iteration of Alg. 4 / Alg. 5 for all right-hand sides, entirely on the device.
// With a preconditioner the operator is D c M: v = D (c M p), t = D (c M s), and (t, s) is
// taken against s itself (the TSAux epilogue), so x accumulates the iterate u of D c M u = y
// (even-odd: the Schur matrix times the even-even block of c M).
void bicg_iteration(const qcd_gauge* g, int prec, double kappa, const Work& w, int ftz, const Precond& pc,
                    hipStream_t st) {
  const Geom& G = g->g;
  const int n = w.n;
  const DslashTune& tu = g->tune[prec];
  const int drows = dslash_partial_rows(G, tu, n), frows = flat_rows(G, prec);
  const void* U = g->U[prec];
  if (w.eo) {  // A = 1 - kappa^2 H_eo H_oe on even-parity fields, two launches per product
    const Geom gh = half_geom(G);
    const int erows = dslash_partial_rows(G, tu, n, true);
    const double k2 = kappa * kappa;
    launch_p_update(gh, prec, n, w.sc, w.p, w.v, w.r, ftz, st);
    const void* pv = w.p;  // the vector the Schur operator acts on: p, or c M p
    if (pc.net) {
      precond_apply(g, pc, w, n, w.p, w.z, ftz, w.sc, st);
      pv = w.z;
    }
    launch_dslash(prec, G, tu, kOpH, kEpiNone, n, w.t1, pv, U, 1.0, nullptr, nullptr, w.sc, ftz, st, nullptr, 1);
    launch_dslash(prec, G, tu, kOpD, kEpiDotAux, n, w.v, w.t1, U, k2, w.rstar, w.partials, w.sc, ftz, st, pv, 0);
    launch_alpha(n, w.sc, w.partials, erows, st);
    launch_s_update(gh, prec, n, w.sc, w.r, w.v, ftz, st);
    if (pc.net) {  // t = A (c M s), with (t, s) taken against s itself
      precond_apply(g, pc, w, n, w.r, w.z, ftz, w.sc, st);
      launch_dslash(prec, G, tu, kOpH, kEpiNone, n, w.t1, w.z, U, 1.0, nullptr, nullptr, w.sc, ftz, st, nullptr, 1);
      launch_dslash(prec, G, tu, kOpD, kEpiTSAux, n, w.t, w.t1, U, k2, w.r, w.partials, w.sc, ftz, st, w.z, 0);
    } else {
      launch_dslash(prec, G, tu, kOpH, kEpiNone, n, w.t1, w.r, U, 1.0, nullptr, nullptr, w.sc, ftz, st, nullptr, 1);
      launch_dslash(prec, G, tu, kOpD, kEpiTS, n, w.t, w.t1, U, k2, nullptr, w.partials, w.sc, ftz, st, w.r, 0);
    }
    launch_omega(n, w.sc, w.partials, erows, st);
    launch_xr_update(gh, prec, n, w.sc, w.x, w.r, w.t, w.p, w.rstar, w.partials, ftz, st);
    launch_iter_end(n, w.sc, w.partials, flat_rows(gh, prec), w.history, w.hist_stride, st);
    return;
  }
  launch_p_update(G, prec, n, w.sc, w.p, w.v, w.r, ftz, st);
  if (pc.net) {
    precond_apply(g, pc, w, n, w.p, w.z, ftz, w.sc, st);
    launch_dslash(prec, G, tu, kOpD, kEpiDotAux, n, w.v, w.z, U, kappa, w.rstar, w.partials, w.sc, ftz, st);
  } else {
    launch_dslash(prec, G, tu, kOpD, kEpiDotAux, n, w.v, w.p, U, kappa, w.rstar, w.partials, w.sc, ftz, st);
  }
  launch_alpha(n, w.sc, w.partials, drows, st);
  launch_s_update(G, prec, n, w.sc, w.r, w.v, ftz, st);
  if (pc.net) {
    precond_apply(g, pc, w, n, w.r, w.z, ftz, w.sc, st);
    launch_dslash(prec, G, tu, kOpD, kEpiTSAux, n, w.t, w.z, U, kappa, w.r, w.partials, w.sc, ftz, st);
  } else {
    launch_dslash(prec, G, tu, kOpD, kEpiTS, n, w.t, w.r, U, kappa, nullptr, w.partials, w.sc, ftz, st);
  }
  launch_omega(n, w.sc, w.partials, drows, st);
  launch_xr_update(G, prec, n, w.sc, w.x, w.r, w.t, w.p, w.rstar, w.partials, ftz, st);
  launch_iter_end(n, w.sc, w.partials, frows, w.history, w.hist_stride, st);
}

// FP64 residual r = b - D x with |r|^2 partials for all right-hand sides
// (only those still refining are computed).
// With outer_mask, only the right-hand sides it selects are computed (mask 1:
// those whose device-driven refinement step is due).
void residual64(const qcd_gauge* g, double kappa, const Work& w, const Scalars* outer_mask, hipStream_t st,
                int mask = 0) {
  if (w.eo) {  // r = b' - (x_e - kappa^2 H_eo H_oe x_e)
    launch_dslash(kFP64, g->g, g->tune[kFP64], kOpH, kEpiNone, w.n, w.t64, w.x64, g->U[kFP64], 1.0, nullptr, nullptr,
                  outer_mask, 0, st, nullptr, 1, mask);
    launch_dslash(kFP64, g->g, g->tune[kFP64], kOpD, kEpiResid, w.n, w.r64, w.t64, g->U[kFP64], kappa * kappa,
                  w.bp64, w.partials, outer_mask, 0, st, w.x64, 0, mask);
    return;
  }
  launch_dslash(kFP64, g->g, g->tune[kFP64], kOpD, kEpiResid, w.n, w.r64, w.x64, g->U[kFP64], kappa, w.b64,
                w.partials, outer_mask, 0, st, nullptr, -1, mask);
}
int residual_rows(const qcd_gauge* g, const Work& w) {
  return dslash_partial_rows(g->g, g->tune[kFP64], w.n, w.eo);
}

// Even-odd set-up: the canonical FP64 source goes straight to eta_e and eta_o
// (|b|^2 partials of the full field, site_grid rows), then the right-hand side
// b' = eta_e + kappa H_eo eta_o of eq. (4)-(6) (D_ee = D_oo = 1, D_eo = -kappa H_eo).
void eo_setup(const qcd_gauge* g, double kappa, const Work& w, const void* b_dev, hipStream_t st) {
  launch_pack_spinor_split(g->g, w.n, w.eta_e, w.eta_o, (const double*)b_dev, w.partials, st);
  launch_dslash(kFP64, g->g, g->tune[kFP64], kOpD, kEpiNone, w.n, w.bp64, w.eta_o, g->U[kFP64], -kappa, nullptr,
                nullptr, nullptr, 0, st, w.eta_e, 0);
}
// x_o = eta_o + kappa H_oe x_e, the canonical solution, and |b - D x|^2 of the
// full system per right-hand side in r2 (synchronises): the odd rows come from
// the reconstruction launch itself; with even_rows the even rows eta_e - (x_e -
// kappa H_eo x_o) from one more one-parity launch (residual vector left in
// r64), else r2 holds the odd rows only (the caller adds the even rows it has).
// With hop_kept, t64 holds H_oe x_e of the x_e returned (the last refinement
// step's residual computed it) and the reconstruction streams instead of hopping.
qcd_status eo_finish(const qcd_gauge* g, double kappa, const Work& w, void* x_dev, double* r2, hipStream_t st,
                     bool even_rows = true, bool hop_kept = false) {
  const Geom& G = g->g;
  const int n = w.n;
  DslashTune one = g->tune[kFP64];
  one.rhs_tile = 1;
  const Geom gh = half_geom(G);
  const int rows_o = hop_kept ? site_grid(gh) : dslash_partial_rows(G, one, n, true);
  const int rows_e = dslash_partial_rows(G, g->tune[kFP64], n, true);
  double* po = w.partials;
  double* pe = w.partials + (size_t)n * rows_o;
  if (hop_kept) {  // x_o goes straight to the canonical output
    launch_eo_recon_unpack(G, n, (double*)x_dev, (const double*)w.x64, (const double*)w.eta_o,
                           (const double*)w.t64, kappa, po, st);
  } else {
    launch_dslash(kFP64, G, g->tune[kFP64], kOpD, kEpiRecon, n, w.x64o, w.x64, g->U[kFP64], -kappa, nullptr, po,
                  nullptr, 0, st, w.eta_o, 1);
    if (even_rows)
      launch_dslash(kFP64, G, g->tune[kFP64], kOpD, kEpiResid, n, w.r64, w.x64o, g->U[kFP64], kappa, w.eta_e, pe,
                    nullptr, 0, st, w.x64, 0);
    launch_unpack_spinor_split(G, n, (double*)x_dev, w.x64, w.x64o, st);
  }
  launch_finish_sum(n, po, rows_o, 1, w.sums, st);
  if (even_rows) launch_finish_sum(n, pe, rows_e, 1, w.sums + n, st);
  HIP_LAUNCHED();
  double h[2 * kMaxRhs];
  HIP_TRY(hipMemcpyAsync(h, w.sums, (even_rows ? 2 : 1) * n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < n; i++) r2[i] = h[i] + (even_rows ? h[n + i] : 0.0);
  return QCD_OK;
}

// The refinement step of Alg. 3 run from the device, for the right-hand sides
// whose inner solve has stopped (every kernel checks outer_step): x += (|r| /
// s^) double(t~), the FP64 residual r = b - D x and its norm (step count,
// stop tests, log), y~ = low(r s / |r|) and s^, and the next inner start.
void device_step(const qcd_gauge* g, double kappa, const Work& w, const qcd_ir_params* p, hipStream_t st) {
  const Geom G = w.eo ? half_geom(g->g) : g->g;  // geometry of the refined vectors
  const int prec = p->inner_prec;
  launch_correct(G, prec, w.n, w.sc, (double*)w.x64, w.x, st);
  residual64(g, kappa, w, w.sc, st, 1);
  launch_outer_residual_norm(w.n, w.sc, w.partials, dslash_partial_rows(g->g, g->tune[kFP64], w.n, w.eo), p->s, st,
                             w.outer_log);
  launch_convert(G, prec, w.n, w.sc, (const double*)w.r64, w.r, w.rstar, w.partials, p->inner.ftz, st);
  launch_convert_finish(w.n, w.sc, w.partials, site_grid(G), p->recalc_shat, p->s, st);
}

// Capture one iteration (8 kernels, 14 with the network; even-odd 10 and 20) into a hip graph.
// Capture runs on the handle's own stream (the null stream cannot be
// captured); the graph is launched on the caller's stream.  The kernels take
// every changing value from device memory, so one capture serves every
// iteration.
qcd_status iteration_graph(const qcd_gauge* gc, int prec, double kappa, const Work& w, int ftz, const Precond& pc,
                           hipGraphExec_t* out) {
  qcd_gauge* g = const_cast<qcd_gauge*>(gc);
  unsigned long long kbits;
  memcpy(&kbits, &kappa, sizeof kbits);
  unsigned sbits;
  memcpy(&sbits, &pc.scale, sizeof sbits);
  // Everything the captured launches bake in: the scalar parameters, the launch
  // shape, and the address of every workspace region they read or write (the
  // regions move when max_iter or nrhs changes the carve of one workspace).
  auto u = [](const void* q) { return (unsigned long long)(uintptr_t)q; };
  const unsigned long long key[32] = {(unsigned long long)prec, (unsigned long long)w.n, kbits,
                                      (unsigned long long)ftz,
                                      ((unsigned long long)(unsigned)g->tune[prec].sched << 16) |
                                          ((unsigned long long)(unsigned)g->tune[prec].variant << 8) |
                                          ((unsigned long long)(g->tune[prec].rhs_tile & 0xff)) |
                                          ((unsigned long long)w.eo << 24) |
                                          ((unsigned long long)(g->tune[kFP64].rhs_tile & 0xff) << 32) |
                                          ((unsigned long long)(unsigned)g->tune[kFP64].sched << 40) |
                                          ((unsigned long long)(unsigned)g->tune[kFP64].variant << 48),
                                      u(pc.net), pc.net ? sbits : 0ull, u(w.x), u(w.r), u(w.rstar), u(w.p), u(w.v),
                                      u(w.t), u(w.z), u(w.t1), u(w.partials), u(w.sc), u(w.history),
                                      (unsigned long long)w.hist_stride, u(w.sums), u(w.scale),
                                      (unsigned long long)w.bytes, u(w.zin), u(w.zout)};
  if (g->graph_exec && memcmp(key, g->graph_key, sizeof key) == 0) {
    *out = g->graph_exec;
    return QCD_OK;
  }
  if (g->graph_exec) {
    HIP_TRY(hipGraphExecDestroy(g->graph_exec));
    g->graph_exec = nullptr;
  }
  hipGraph_t graph;
  HIP_TRY(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
  bicg_iteration(g, prec, kappa, w, ftz, pc, g->cap_stream);
  hipError_t e = hipStreamEndCapture(g->cap_stream, &graph);
  if (e != hipSuccess) return fail(QCD_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g->graph_exec = nullptr;
    return fail(QCD_ERR_HIP, "graph instantiation: %s", hipGetErrorString(e));
  }
  memcpy(g->graph_key, key, sizeof key);
  *out = g->graph_exec;
  return QCD_OK;
}

bool any_active(const qcd_gauge* g, int n) {
  for (int i = 0; i < n; i++)
    if (g->host_sc[i].active) return true;
  return false;
}

// One inner solve in progress: a handle, its workspace and its preconditioner.
struct InnerRun {
  const qcd_gauge* g;
  int prec;
  double kappa;
  const Work* w;
  Precond pc;
};

// Copy every run's device scalars to its handle's host mirror, one synchronisation.
qcd_status read_scalars_all(const InnerRun* runs, int nrun, hipStream_t st) {
  for (int r = 0; r < nrun; r++)
    HIP_TRY(hipMemcpyAsync(runs[r].g->host_sc, runs[r].w->sc, sizeof(Scalars) * runs[r].w->n, hipMemcpyDeviceToHost,
                           st));
  HIP_TRY(hipStreamSynchronize(st));
  return QCD_OK;
}

// Run the inner loops of several solves (one per run) from initialised
// scalars until the device reports a stop for every right-hand side of every
// run; fills the host mirrors.  Iterations are queued in chunks without host
// synchronisation (kernels of a stopped solve return at once).  After the
// first chunk, the chunk length is the number of iterations the observed
// convergence rate predicts the slowest right-hand side still needs, plus
// one.  With several runs each chunk forks from st onto every run's own
// stream (runs on different lattices proceed concurrently) and joins back.
// Without entry_read the first chunk is queued for every right-hand side the
// host mirror shows as refining (outer_active), without a synchronisation;
// the kernels skip those the device has already stopped.
qcd_status bicg_loop_multi(const InnerRun* runs, int nrun, const qcd_bicgstab_params& p, hipStream_t st,
                           bool entry_read = true) {
  const int K0 = p.check_every > 0 ? p.check_every : 4;
  qcd_status s = QCD_OK;
  if (entry_read) {
    if ((s = read_scalars_all(runs, nrun, st))) return s;
  } else {
    for (int r = 0; r < nrun; r++)
      for (int i = 0; i < runs[r].w->n; i++) runs[r].g->host_sc[i].active = runs[r].g->host_sc[i].outer_active;
  }
  std::vector<hipGraphExec_t> gexec(nrun, nullptr);
  std::vector<hipStream_t> rs(nrun, st);
  // several runs: each on its handle's own stream, forked from st by the first
  // handle's fork event and joined by each handle's done event (all created at
  // upload, so a solve creates no HIP objects)
  hipEvent_t fork = runs[0].g->ev_fork;
  for (int r = 0; r < nrun; r++) {
    qcd_gauge* g = const_cast<qcd_gauge*>(runs[r].g);
    if (p.use_graph && any_active(g, runs[r].w->n))
      if ((s = iteration_graph(g, runs[r].prec, runs[r].kappa, *runs[r].w, p.ftz, runs[r].pc, &gexec[r]))) return s;
    if (nrun > 1) rs[r] = g->cap_stream;
  }
  auto anyrun = [&]() {
    for (int r = 0; r < nrun; r++)
      if (any_active(runs[r].g, runs[r].w->n)) return true;
    return false;
  };
  // residual^2 at the last poll (at iteration 0: |b|^2, set when the run started)
  std::vector<double> prev_res2((size_t)nrun * kMaxRhs);
  std::vector<int> prev_iter((size_t)nrun * kMaxRhs, 0);
  int launched = 0, chunk = K0;
  while (anyrun() && launched <= p.max_iter + K0) {
    if (nrun > 1) HIP_TRY(hipEventRecord(fork, st));
    for (int r = 0; r < nrun; r++) {
      const InnerRun& R = runs[r];
      if (!any_active(R.g, R.w->n)) continue;
      if (nrun > 1) HIP_TRY(hipStreamWaitEvent(rs[r], fork, 0));
      for (int j = 0; j < chunk; j++) {
        if (gexec[r])
          HIP_TRY(hipGraphLaunch(gexec[r], rs[r]));
        else
          bicg_iteration(R.g, R.prec, R.kappa, *R.w, p.ftz, R.pc, rs[r]);
      }
      if (nrun > 1) {
        HIP_TRY(hipEventRecord(R.g->ev_done, rs[r]));
        HIP_TRY(hipStreamWaitEvent(st, R.g->ev_done, 0));
      }
    }
    HIP_LAUNCHED();
    launched += chunk;
    if ((s = read_scalars_all(runs, nrun, st))) return s;
    chunk = K0;
    if (p.check_every > 0) continue;
    int need_max = 0;
    for (int r = 0; r < nrun; r++)
      for (int i = 0; i < runs[r].w->n; i++) {
        const Scalars& h = runs[r].g->host_sc[i];
        double& pr = prev_res2[(size_t)r * kMaxRhs + i];
        int& pi = prev_iter[(size_t)r * kMaxRhs + i];
        if (!h.active || h.iter <= pi) continue;
        if (pi == 0) pr = h.bnorm2;
        const double res2 = h.rnorm2 / (h.gamma_cum * h.gamma_cum);
        const double target = h.tol2 * h.bnorm2;
        const double rate = std::pow(res2 / pr, 1.0 / (h.iter - pi));  // per iteration
        int need = K0;
        if (rate > 0.0 && rate < 0.999 && res2 > target)
          need = (int)std::min(64.0, std::max(1.0, std::ceil(std::log(target / res2) / std::log(rate)) + 1.0));
        need_max = std::max(need_max, need);
        pr = res2;
        pi = h.iter;
      }
    if (need_max > 0) chunk = need_max;
  }
  return QCD_OK;
}

qcd_status bicg_loop(const qcd_gauge* g, int prec, double kappa, const Work& w, const qcd_bicgstab_params& p,
                     const Precond& pc, hipStream_t st) {
  const InnerRun run{g, prec, kappa, &w, pc};
  return bicg_loop_multi(&run, 1, p, st);
}

void copy_history(qcd_solve_info* info, const Work& w, int rhs, int niter, double bn2, hipStream_t st) {
  if (!info || !info->history || info->history_cap <= info->history_len || niter <= 0) return;
  int m = niter;
  if (m > info->history_cap - info->history_len) m = info->history_cap - info->history_len;
  if (hipMemcpyAsync(info->history + info->history_len, w.history + (size_t)rhs * w.hist_stride, m * sizeof(double),
                     hipMemcpyDeviceToHost, st) != hipSuccess)
    return;
  if (hipStreamSynchronize(st) != hipSuccess) return;
  for (int i = 0; i < m; i++) info->history[info->history_len + i] /= bn2;
  info->history_len += m;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

const char* qcd_last_error(void) { return g_err.c_str(); }

qcd_status qcd_gauge_upload(qcd_gauge** out, const int dims[4], const void* U_dev, int prec_mask, void* stream) {
  if (!out || !dims || !U_dev) return fail(QCD_ERR_ARG, "null argument");
  for (int i = 0; i < 4; i++)
    if (dims[i] < 2 || dims[i] % 2) return fail(QCD_ERR_ARG, "extent %d of direction %d must be even and >= 2", dims[i], i);
  const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
  if (V / 2 >= (1ll << 30)) return fail(QCD_ERR_ARG, "lattice too large");
  const int flags = prec_mask & ~15;
  prec_mask &= 15;
  if (prec_mask == 0) prec_mask = 15;
  prec_mask |= 1 << kFP64;
  qcd_gauge* g = new qcd_gauge();
  memset(g, 0, sizeof(*g));
  g->g = make_geom(dims);
  {  // the static workspace's address on this device, once per device
    void* sp = nullptr;
    const qcd_status src = scratch_address(&sp);
    if (src != QCD_OK) {
      delete g;
      return src;
    }
  }
  // defaults measured on MI355X at 32^3 x 64 with rotating buffers and in the
  // even-odd solves (the tuner may override them): z slabs per XCD; prefetch 2
  // hops at 2 waves per SIMD (FP16 and FP32 with their x and y neighbours
  // staged in LDS where the form applies: FP16 in the full-lattice and the
  // one-parity launches, FP32 in the one-parity ones), 1 hop at 2 (FP64, whose
  // LDS form measured no faster)
  g->tune[kFP64] = DslashTune{1, 0, 0, 0};
  g->tune[kFP32] = DslashTune{1, 6, 0, 0};
  g->tune[kFP16] = DslashTune{1, 6, 0, 0};
  g->tune[kBF16] = DslashTune{1, 1, 0, 0};
  memcpy(g->dims, dims, sizeof g->dims);
  hipStream_t st = S(stream);
  qcd_status rc = QCD_OK;
  // Links whose row 2 equals conj(row0 x row1) to within the rounding of a
  // precision are stored as rows 0 and 1 only in that precision.
  g->su3_dev = INFINITY;
  if (!(flags & QCD_LINKS_FULL)) {
    const int rows = site_grid(g->g);
    double* part = nullptr;
    if (hipMalloc(&part, (rows + 1) * sizeof(double)) != hipSuccess) {
      delete g;
      return fail(QCD_ERR_HIP, "hipMalloc failed");
    }
    launch_link_su3_dev(g->g, (const double*)U_dev, part, part + rows, st);
    hipError_t e = hipMemcpyAsync(&g->su3_dev, part + rows, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) {
      delete g;
      return fail(QCD_ERR_HIP, "link check failed: %s", hipGetErrorString(e));
    }
    const double thr[kNumPrec] = {1e-14, 1e-7, 1e-4, 1e-3};
    for (int p = 0; p < kNumPrec; p++) g->tune[p].recon = g->su3_dev <= thr[p];
  }
  for (int p = 0; p < kNumPrec && rc == QCD_OK; p++) {
    if (!(prec_mask & (1 << p))) continue;
    size_t bytes = link_elems(g->g, g->tune[p].recon ? 6 : 9) * prec_complex_bytes(p);
    if (hipMalloc(&g->U[p], bytes) != hipSuccess) {
      g->U[p] = nullptr;
      rc = fail(QCD_ERR_HIP, "hipMalloc of %zu bytes for links failed", bytes);
      break;
    }
    // the padding of the last 64-site block stays zero
    if (hipMemsetAsync(g->U[p], 0, bytes, st) != hipSuccess) rc = fail(QCD_ERR_HIP, "hipMemsetAsync failed");
    launch_pack_links(g->g, p, g->U[p], (const double*)U_dev, g->tune[p].recon, st);
    if (hipGetLastError() != hipSuccess) rc = fail(QCD_ERR_HIP, "link packing launch failed");
  }
  if (rc == QCD_OK && hipHostMalloc((void**)&g->host_sc, sizeof(Scalars) * kMaxRhs, 0) != hipSuccess)
    rc = fail(QCD_ERR_HIP, "hipHostMalloc failed");
  if (rc == QCD_OK &&
      hipHostMalloc((void**)&g->host_log, sizeof(double) * 2 * kOuterLog * kMaxRhs, 0) != hipSuccess)
    rc = fail(QCD_ERR_HIP, "hipHostMalloc failed");
  // the handle's stream (graph capture, batched solves) and its two events:
  // created here so that no solve creates HIP objects
  if (rc == QCD_OK && hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) != hipSuccess)
    rc = fail(QCD_ERR_HIP, "hipStreamCreateWithFlags failed");
  if (rc == QCD_OK && (hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&g->ev_done, hipEventDisableTiming) != hipSuccess))
    rc = fail(QCD_ERR_HIP, "hipEventCreateWithFlags failed");
  if (rc == QCD_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(QCD_ERR_HIP, "synchronise failed");
  if (rc != QCD_OK) {
    qcd_gauge_free(g);
    return rc;
  }
  *out = g;
  return QCD_OK;
}

qcd_status qcd_gauge_free(qcd_gauge* g) {
  if (!g) return QCD_OK;
  for (int p = 0; p < kNumPrec; p++)
    if (g->U[p]) (void)hipFree(g->U[p]);
  if (g->ws) (void)hipFree(g->ws);
  if (g->host_sc) (void)hipHostFree(g->host_sc);
  if (g->host_log) (void)hipHostFree(g->host_log);
  if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  if (g->ev_done) (void)hipEventDestroy(g->ev_done);
  delete g;
  return QCD_OK;
}

qcd_status qcd_set_dslash_tuning(qcd_gauge* g, qcd_prec prec, int sched, int variant, int rhs_tile) {
  if (!g || !valid_prec(prec)) return fail(QCD_ERR_ARG, "invalid handle or precision");
  if (sched < 0 || sched >= kDslashScheds || variant < 0 || variant >= kDslashVariants)
    return fail(QCD_ERR_ARG, "sched must be 0..%d and variant 0..%d", kDslashScheds - 1, kDslashVariants - 1);
  if (rhs_tile != 0 && rhs_tile != 1 && rhs_tile != 2 && rhs_tile != 4 && !(rhs_tile >= -4 && rhs_tile <= -2) &&
      rhs_tile != kRhsTileMfma)
    return fail(QCD_ERR_ARG, "rhs_tile must be 0 (automatic), 1, 2, 4 (lanes), -2, -3, -4 (per thread) or 8 (matrix cores)");
  g->tune[prec] = DslashTune{sched, variant, rhs_tile, g->tune[prec].recon};
  return QCD_OK;
}

int qcd_gauge_link_reals(const qcd_gauge* g, qcd_prec prec) {
  if (!g || !valid_prec(prec) || !g->U[prec]) return 0;
  return g->tune[prec].recon ? 12 : 18;
}

qcd_status qcd_get_dslash_tuning(const qcd_gauge* g, qcd_prec prec, int* sched, int* variant, int* rhs_tile) {
  if (!g || !valid_prec(prec) || !sched || !variant || !rhs_tile) return fail(QCD_ERR_ARG, "invalid argument");
  *sched = g->tune[prec].sched;
  *variant = g->tune[prec].variant;
  *rhs_tile = g->tune[prec].rhs_tile;
  return QCD_OK;
}

// Autotuner: time every launch choice of the Wilson operator for (prec,
// nrhs) on scratch fields with HIP events and keep the fastest.  With a cache
// path, results are read from / appended to a JSON-lines file keyed by
// lattice, precision, number of right-hand sides and GPU architecture.
qcd_status qcd_autotune_dslash(qcd_gauge* g, qcd_prec prec, int nrhs, int reps, const char* cache_path,
                               double* best_us, void* stream) {
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (reps < 1) reps = 20;
  hipDeviceProp_t prop;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  char arch[64];
  snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  for (char* c = arch; *c; c++)
    if (*c == ':') { *c = 0; break; }
  char key[256];
  snprintf(key, sizeof key, "\"dims\": \"%dx%dx%dx%d\", \"prec\": %d, \"nrhs\": %d, \"links\": %d, \"arch\": \"%s\"",
           g->dims[0], g->dims[1], g->dims[2], g->dims[3], (int)prec, nrhs, g->tune[prec].recon ? 12 : 18, arch);
  if (cache_path && cache_path[0]) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[1024];
      while (fgets(line, sizeof line, f)) {
        if (!strstr(line, key)) continue;
        int sc = -1, va = -1, rt = -1;
        double us = 0;
        const char* q = strstr(line, "\"sched\":");
        if (q) sscanf(q, "\"sched\": %d, \"variant\": %d, \"rhs_tile\": %d, \"us\": %lf", &sc, &va, &rt, &us);
        if (sc >= 0 && va >= 0 && rt >= 0) {
          fclose(f);
          g->tune[prec] = DslashTune{sc, va, rt, g->tune[prec].recon};
          if (best_us) *best_us = us;
          return QCD_OK;
        }
      }
      fclose(f);
    }
  }
  hipStream_t st = S(stream);
  const size_t bytes = (size_t)nrhs * spinor_bytes(g->g, prec);
  // Rotate input/output pairs whose total exceeds the last-level cache
  // (256 MB on MI355X), as the vectors of a solve do; a single pair would stay
  // cache-resident and favour the wrong launch shape.
  const int npair = (int)std::min<size_t>(4, std::max<size_t>(1, ((size_t)512 << 20) / (2 * bytes) + 1));
  void* buf[8] = {};
  for (int i = 0; i < 2 * npair; i++) {
    if (hipMalloc(&buf[i], bytes) != hipSuccess) {
      for (int j = 0; j < i; j++) (void)hipFree(buf[j]);
      return fail(QCD_ERR_HIP, "hipMalloc failed");
    }
    // finite, normal values in every precision (bytes 0x3c)
    (void)hipMemsetAsync(buf[i], 0x3c, bytes, st);
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  DslashTune best = g->tune[prec];
  float best_ms = 1e30f;
  const int tiles[7] = {1, 2, 4, -2, -3, -4, kRhsTileMfma};
  for (int ti = 0; ti < 7; ti++) {
    const int T = tiles[ti];
    const int A = T < 0 ? -T : T;
    if (T == kRhsTileMfma) {
      if (prec != QCD_FP16 || mfma_rhs_tile(nrhs) == 0) continue;
    } else if (nrhs % A || (A > 1 && nrhs == 1)) {
      continue;
    }
    for (int sched = 0; sched < (T == kRhsTileMfma ? 1 : kDslashScheds); sched++)
      for (int var = 0; var < (T == 1 ? kDslashVariants : 1); var++) {
        if (sched > 1 && make_sched(g->g, sched, T > 0 ? T : 1, T > 0 ? nrhs : nrhs / A).mode != sched)
          continue;  // not applicable
        const DslashTune tu{sched, var, T, g->tune[prec].recon};
        for (int i = 0; i < 2; i++)
          launch_dslash(prec, g->g, tu, kOpD, kEpiNone, nrhs, buf[2 * (i % npair) + 1], buf[2 * (i % npair)],
                        g->U[prec], 0.1, nullptr, nullptr, nullptr, 0, st);
        (void)hipEventRecord(e0, st);
        for (int i = 0; i < reps; i++)
          launch_dslash(prec, g->g, tu, kOpD, kEpiNone, nrhs, buf[2 * (i % npair) + 1], buf[2 * (i % npair)],
                        g->U[prec], 0.1, nullptr, nullptr, nullptr, 0, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_ms) {
          best_ms = ms;
          best = tu;
        }
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int i = 0; i < 2 * npair; i++) (void)hipFree(buf[i]);
  HIP_LAUNCHED();
  g->tune[prec] = best;
  if (best_us) *best_us = best_ms * 1e3;
  if (cache_path && cache_path[0]) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "{%s, \"sched\": %d, \"variant\": %d, \"rhs_tile\": %d, \"us\": %.3f}\n", key, best.sched,
              best.variant, best.rhs_tile, best_ms * 1e3);
      fclose(f);
    }
  }
  return QCD_OK;
}

size_t qcd_spinor_bytes(const qcd_gauge* g, qcd_prec prec) {
  if (!g || !valid_prec(prec)) return 0;
  return spinor_bytes(g->g, prec);
}

size_t qcd_workspace_bytes(const qcd_gauge* g, int what, qcd_prec prec, int max_iter, int nrhs) {
  if (!g || !valid_prec(prec) || (what & ~(7 | kWhatEO)) || (what & 7) > 3 || nrhs < 1 || nrhs > kMaxRhs) return 0;
  if ((what & kWhatEO) && (what & 7) == 2) return 0;
  return carve(g, what, prec, max_iter, nrhs, nullptr).bytes;
}

qcd_status qcd_convert(const qcd_gauge* g, qcd_prec prec, int nrhs, void* native_dev, const void* canonical_dev,
                       double scale, int ftz, double* norm2, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!valid_prec(prec) || !native_dev || !canonical_dev) return fail(QCD_ERR_ARG, "invalid argument");
  if ((rc = check_canonical(canonical_dev, "canonical field"))) return rc;
  hipStream_t st = S(stream);
  Work w;
  if (norm2) {
    rc = get_work(g, 2, prec, 0, nrhs, nullptr, 0, &w);
    if (rc) return rc;
  }
  launch_pack_spinor(g->g, prec, nrhs, native_dev, (const double*)canonical_dev, scale, ftz,
                     norm2 ? w.partials : nullptr, st);
  HIP_LAUNCHED();
  if (norm2) return read_sum(w, site_grid(g->g), 1, norm2, st);
  return QCD_OK;
}

qcd_status qcd_unconvert(const qcd_gauge* g, qcd_prec prec, int nrhs, void* canonical_dev, const void* native_dev,
                         double scale, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!valid_prec(prec) || !native_dev || !canonical_dev) return fail(QCD_ERR_ARG, "invalid argument");
  if ((rc = check_canonical(canonical_dev, "canonical field"))) return rc;
  launch_unpack_spinor(g->g, prec, nrhs, (double*)canonical_dev, native_dev, nullptr, scale, S(stream));
  HIP_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_gaussian_spinors(void* out_dev, int64_t ncomplex, uint64_t seed, void* stream) {
  if (!out_dev || ncomplex < 0) return fail(QCD_ERR_ARG, "invalid argument");
  if (ncomplex == 0) return QCD_OK;
  launch_gaussian((double*)out_dev, ncomplex, seed, S(stream));
  HIP_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_dslash(const qcd_gauge* g, double kappa, qcd_op op, qcd_prec prec, qcd_layout layout, int nrhs,
                      void* out_dev, const void* in_dev, void* stream) {
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!out_dev || !in_dev || out_dev == in_dev) return fail(QCD_ERR_ARG, "out and in must be distinct non-null buffers");
  if (op < QCD_OP_D || op > QCD_OP_SCHUR) return fail(QCD_ERR_ARG, "invalid op %d", (int)op);
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if (layout == QCD_LAYOUT_CANONICAL &&
      ((rc = check_canonical(out_dev, "out")) || (rc = check_canonical(in_dev, "in"))))
    return rc;
  hipStream_t st = S(stream);
  if (op == QCD_OP_SCHUR) {
    // out_e = in_e - kappa^2 H_eo H_oe in_e, out_o = 0; the odd half of out holds H_oe in_e meanwhile
    const void* src = in_dev;
    void* dst = out_dev;
    Work w;
    if (layout == QCD_LAYOUT_CANONICAL) {
      if ((rc = get_work(g, 2, prec, 0, nrhs, nullptr, 0, &w))) return rc;
      launch_pack_spinor(g->g, prec, nrhs, w.x, (const double*)in_dev, 1.0, 0, nullptr, st);
      src = w.x;
      dst = w.r;
    } else if (layout != QCD_LAYOUT_NATIVE) {
      return fail(QCD_ERR_ARG, "invalid layout");
    }
    const Geom gh = half_geom(g->g);
    const size_t full = spinor_bytes(g->g, prec), half = spinor_bytes(gh, prec);
    for (int r = 0; r < nrhs; r++) {
      const char* xe = (const char*)src + r * full;
      char* ye = (char*)dst + r * full;
      launch_dslash(prec, g->g, g->tune[prec], kOpH, kEpiNone, 1, ye + half, xe, g->U[prec], 1.0, nullptr, nullptr,
                    nullptr, 0, st, nullptr, 1);
      launch_dslash(prec, g->g, g->tune[prec], kOpD, kEpiNone, 1, ye, ye + half, g->U[prec], kappa * kappa, nullptr,
                    nullptr, nullptr, 0, st, xe, 0);
      launch_zero(gh, prec, 1, ye + half, st);
    }
    if (layout == QCD_LAYOUT_CANONICAL) launch_unpack_spinor(g->g, prec, nrhs, (double*)out_dev, w.r, nullptr, 1.0, st);
    HIP_LAUNCHED();
    return QCD_OK;
  }
  if (layout == QCD_LAYOUT_NATIVE) {
    launch_dslash(prec, g->g, g->tune[prec], op, kEpiNone, nrhs, out_dev, in_dev, g->U[prec], kappa, nullptr, nullptr,
                  nullptr, 0, st);
    HIP_LAUNCHED();
    return QCD_OK;
  }
  if (layout != QCD_LAYOUT_CANONICAL) return fail(QCD_ERR_ARG, "invalid layout");
  Work w;
  rc = get_work(g, 2, prec, 0, nrhs, nullptr, 0, &w);
  if (rc) return rc;
  launch_pack_spinor(g->g, prec, nrhs, w.x, (const double*)in_dev, 1.0, 0, nullptr, st);
  launch_dslash(prec, g->g, g->tune[prec], op, kEpiNone, nrhs, w.r, w.x, g->U[prec], kappa, nullptr, nullptr, nullptr,
                0, st);
  launch_unpack_spinor(g->g, prec, nrhs, (double*)out_dev, w.r, nullptr, 1.0, st);
  HIP_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_residual(const qcd_gauge* g, double kappa, int nrhs, void* r_dev, const void* x_dev, const void* b_dev,
                        double* norm2, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!r_dev || !x_dev || !b_dev) return fail(QCD_ERR_ARG, "null argument");
  if ((rc = check_canonical(r_dev, "r")) || (rc = check_canonical(x_dev, "x")) || (rc = check_canonical(b_dev, "b")))
    return rc;
  hipStream_t st = S(stream);
  Work w;
  rc = get_work(g, 1, kFP64, 1, nrhs, nullptr, 0, &w);
  if (rc) return rc;
  launch_pack_spinor(g->g, kFP64, nrhs, w.x64, (const double*)x_dev, 1.0, 0, nullptr, st);
  launch_pack_spinor(g->g, kFP64, nrhs, w.b64, (const double*)b_dev, 1.0, 0, nullptr, st);
  residual64(g, kappa, w, nullptr, st);
  launch_unpack_spinor(g->g, kFP64, nrhs, (double*)r_dev, w.r64, nullptr, 1.0, st);
  HIP_LAUNCHED();
  if (norm2) return read_sum(w, dslash_partial_rows(g->g, g->tune[kFP64], nrhs), 1, norm2, st);
  return QCD_OK;
}

static qcd_status status_of(int s, int iters) {
  switch (s) {
    case kConverged: return QCD_OK;
    case kMaxIter: return QCD_NOT_CONVERGED;
    case kBreakdown: return fail(QCD_ERR_BREAKDOWN, "BiCGStab breakdown after %d iterations", iters);
    case kNonFinite: return fail(QCD_ERR_NONFINITE, "non-finite solver scalar after %d iterations", iters);
    default: return fail(QCD_ERR_HIP, "solver stopped in an unknown state %d", s);
  }
}

// worst of two statuses: errors (negative) beat warnings beat QCD_OK
static qcd_status worse(qcd_status a, qcd_status b) {
  if (a < 0 || b < 0) return a < b ? a : b;
  return a > b ? a : b;
}

}  // extern "C"

namespace {
// Even-odd BiCGStab (eq. (4)-(6)): b' = eta_e + kappa H_eo eta_o in FP64,
// Alg. 4 / 5 on A = 1 - kappa^2 H_eo H_oe in precision prec, then
// x_o = eta_o + kappa H_oe x_e in FP64; the reported residual is the full
// |b - D x| / |b|.
qcd_status bicgstab_eo(const qcd_gauge* g, double kappa, int prec, int n, void* x_dev, const void* b_dev,
                       const qcd_bicgstab_params& p, qcd_solve_info* info, const Work& w, hipStream_t st, double t0) {
  const Geom& G = g->g;
  const Geom gh = half_geom(G);
  qcd_status rc;
  Scalars hs[kMaxRhs];
  for (int i = 0; i < n; i++) init_params(&hs[i], p);
  HIP_TRY(hipMemcpyAsync(w.sc, hs, sizeof(Scalars) * n, hipMemcpyHostToDevice, st));
  double b2[kMaxRhs], r2[kMaxRhs];
  eo_setup(g, kappa, w, b_dev, st);
  if ((rc = read_sum(w, site_grid(G), 1, b2, st))) return rc;
  // r = r* = low(b'), x0 = 0
  launch_narrow(gh, prec, n, w.r, (const double*)w.bp64, w.partials, p.ftz, st);
  HIP_TRY(hipMemcpyAsync(w.rstar, w.r, n * spinor_bytes(gh, prec), hipMemcpyDeviceToDevice, st));
  launch_bicg_init(n, w.sc, w.partials, site_grid(gh), st);
  HIP_LAUNCHED();
  if ((rc = bicg_loop(g, prec, kappa, w, p, Precond{}, st))) return rc;
  Scalars sc[kMaxRhs];
  memcpy(sc, g->host_sc, sizeof(Scalars) * n);
  double scales[kMaxRhs];
  for (int i = 0; i < n; i++) {
    scales[i] = sc[i].iter > 0 ? sc[i].xscale / sc[i].lambda_cum : 0.0;
    if (sc[i].iter == 0) launch_zero(gh, prec, 1, (char*)w.x + i * spinor_bytes(gh, prec), st);
  }
  HIP_TRY(hipMemcpyAsync(w.scale, scales, sizeof(double) * n, hipMemcpyHostToDevice, st));
  launch_widen(gh, prec, n, (double*)w.x64, w.x, w.scale, st);
  if ((rc = eo_finish(g, kappa, w, x_dev, r2, st))) return rc;
  qcd_status result = QCD_OK;
  for (int i = 0; i < n; i++) {
    if (info) {
      qcd_solve_info* in = info + i;
      in->outer_iters = 0;
      in->inner_iters = sc[i].iter;
      in->matvec_low = 2 * sc[i].iter;
      in->matvec_fp64 = 1;
      in->true_rel_residual = b2[i] > 0 ? sqrt(r2[i] / b2[i]) : 0.0;
      in->inner_status = sc[i].status;
      in->first_shat_over_s = 1.0;
      in->history_len = 0;
      copy_history(in, w, i, sc[i].iter, sc[i].bnorm2, st);
      in->seconds = now_s() - t0;
    }
    result = worse(result, status_of(sc[i].status, sc[i].iter));
  }
  return result;
}
}  // namespace

extern "C" {

qcd_status qcd_bicgstab(const qcd_gauge* g, double kappa, qcd_prec prec, int nrhs, void* x_dev, const void* b_dev,
                        const qcd_bicgstab_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const double t0 = now_s();
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!x_dev || !b_dev) return fail(QCD_ERR_ARG, "null vector");
  if ((rc = check_canonical(x_dev, "x")) || (rc = check_canonical(b_dev, "b"))) return rc;
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if ((rc = check_bicg_params(p))) return rc;
  hipStream_t st = S(stream);
  Work w;
  const bool eo = p->even_odd != 0;
  if ((rc = get_work(g, eo ? (1 | kWhatEO) : 1, prec, p->max_iter, nrhs, ws, ws_bytes, &w))) return rc;
  if (eo) return bicgstab_eo(g, kappa, prec, nrhs, x_dev, b_dev, *p, info, w, st, t0);
  const Geom& G = g->g;
  const int n = nrhs;
  const int rows = site_grid(G);
  Scalars hs[kMaxRhs];
  for (int i = 0; i < n; i++) init_params(&hs[i], *p);
  HIP_TRY(hipMemcpyAsync(w.sc, hs, sizeof(Scalars) * n, hipMemcpyHostToDevice, st));
  // r = r* = low(b), x0 = 0
  launch_pack_spinor(G, prec, n, w.r, (const double*)b_dev, 1.0, p->ftz, w.partials, st);
  HIP_TRY(hipMemcpyAsync(w.rstar, w.r, n * spinor_bytes(G, prec), hipMemcpyDeviceToDevice, st));
  launch_bicg_init(n, w.sc, w.partials, rows, st);
  HIP_LAUNCHED();
  if ((rc = bicg_loop(g, prec, kappa, w, *p, Precond{}, st))) return rc;
  Scalars sc[kMaxRhs];
  memcpy(sc, g->host_sc, sizeof(Scalars) * n);
  // x = xscale X / lambda' (zero for a right-hand side that made no step)
  double scales[kMaxRhs];
  for (int i = 0; i < n; i++) {
    scales[i] = sc[i].iter > 0 ? sc[i].xscale / sc[i].lambda_cum : 0.0;
    if (sc[i].iter == 0)  // x of a right-hand side without a step was never written
      launch_zero(G, prec, 1, (char*)w.x + i * spinor_bytes(G, prec), st);
  }
  HIP_TRY(hipMemcpyAsync(w.scale, scales, sizeof(double) * n, hipMemcpyHostToDevice, st));
  launch_unpack_spinor(G, prec, n, (double*)x_dev, w.x, w.scale, 1.0, st);
  HIP_LAUNCHED();
  // FP64 true residual of the returned solutions
  double r2[kMaxRhs], b2[kMaxRhs];
  launch_pack_spinor(G, kFP64, n, w.b64, (const double*)b_dev, 1.0, 0, w.partials, st);
  if ((rc = read_sum(w, rows, 1, b2, st))) return rc;
  launch_pack_spinor(G, kFP64, n, w.x64, (const double*)x_dev, 1.0, 0, nullptr, st);
  residual64(g, kappa, w, nullptr, st);
  if ((rc = read_sum(w, dslash_partial_rows(G, g->tune[kFP64], n), 1, r2, st))) return rc;
  qcd_status result = QCD_OK;
  for (int i = 0; i < n; i++) {
    if (info) {
      qcd_solve_info* in = info + i;
      in->outer_iters = 0;
      in->inner_iters = sc[i].iter;
      in->matvec_low = 2 * sc[i].iter;
      in->matvec_fp64 = 1;
      in->true_rel_residual = b2[i] > 0 ? sqrt(r2[i] / b2[i]) : 0.0;
      in->inner_status = sc[i].status;
      in->first_shat_over_s = 1.0;
      in->history_len = 0;
      copy_history(in, w, i, sc[i].iter, sc[i].bnorm2, st);
      in->seconds = now_s() - t0;
    }
    result = worse(result, status_of(sc[i].status, sc[i].iter));
  }
  return result;
}

}  // extern "C"

namespace {

// One lattice's refinement (Alg. 3) in progress.
struct IrRun {
  const qcd_gauge* g = nullptr;
  double kappa = 0;
  int n = 0;
  void* x_dev = nullptr;
  const void* b_dev = nullptr;
  qcd_solve_info* info = nullptr;
  qcd_ptc* net = nullptr;
  Work w;
  Precond pc;
  double bn[kMaxRhs], rn[kMaxRhs];
  int outer[kMaxRhs], inner_total[kMaxRhs], last_status[kMaxRhs];
  qcd_status result[kMaxRhs];
  bool inner_failed[kMaxRhs];
  Scalars sc[kMaxRhs];  // snapshot after an inner solve
  bool any = false;
  int pc_steps = 0, pc_fallback = -1;
  double bfull[kMaxRhs];  // |b| of the full system (even-odd: the stop test is scaled to it)
  bool log_pending = false;  // the device step log is on its way to the handle's pinned copy
};

qcd_status check_ir_run(const IrRun& R, const qcd_ir_params* p) {
  qcd_status rc = check_gauge(R.g, p->inner_prec);
  if (rc) return rc;
  if ((rc = check_nrhs(R.n))) return rc;
  if (!R.x_dev || !R.b_dev) return fail(QCD_ERR_ARG, "null vector");
  if ((rc = check_canonical(R.x_dev, "x")) || (rc = check_canonical(R.b_dev, "b"))) return rc;
  if (!(R.kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if (R.net) {
    if (p->inner_prec != kFP16) return fail(QCD_ERR_UNSUPPORTED, "the network preconditioner runs with the FP16 inner solve");
    if (ptc_gauge(R.net) != R.g) return fail(QCD_ERR_ARG, "the network is bound to another gauge handle");
    if (!(p->precond_scale >= 0) || !std::isfinite(p->precond_scale))
      return fail(QCD_ERR_ARG, "precond_scale must be finite and >= 0");
  }
  return QCD_OK;
}

// b in the native FP64 layout; r = b, x = 0; |b| and the first rescaling on the device.
// dev: the device-driven refinement follows, whose start (|b|, the even-odd
// tolerance, the step bookkeeping) stays on the device with no host read.
qcd_status ir_start(IrRun& R, const qcd_ir_params* p, hipStream_t st, bool dev) {
  const Geom& G = R.g->g;
  Scalars hs[kMaxRhs];
  for (int i = 0; i < R.n; i++) {
    init_params(&hs[i], p->inner);
    hs[i].out_tol = p->tol;
  }
  HIP_TRY(hipMemcpyAsync(R.w.sc, hs, sizeof(Scalars) * R.n, hipMemcpyHostToDevice, st));
  if (R.w.eo) {
    // eta_e, eta_o and b' (eq. (4)-(6)), |b| of the full system, r = b', x_e = 0
    eo_setup(R.g, R.kappa, R.w, R.b_dev, st);
    if (dev) {
      launch_finish_sum(R.n, R.w.partials, site_grid(G), 1, R.w.sums, st);  // |b|^2, kept on the device
    } else {
      double b2[kMaxRhs];
      qcd_status rc = read_sum(R.w, site_grid(G), 1, b2, st);
      if (rc) return rc;
      for (int i = 0; i < R.n; i++) R.bfull[i] = sqrt(b2[i]);
    }
    const Geom gh = half_geom(G);
    launch_narrow(gh, kFP64, R.n, R.w.r64, (const double*)R.w.bp64, R.w.partials, 0, st);
    launch_outer_residual_norm(R.n, R.w.sc, R.w.partials, site_grid(gh), p->s, st);
    launch_zero(gh, kFP64, R.n, R.w.x64, st);
    if (R.net) launch_zero(G, kFP16, R.n, R.w.zin, st);  // the odd halves the network reads stay zero
    if (dev) launch_ir_dev_start(R.n, R.w.sc, R.w.sums, p->tol, p->max_outer, st);
    return QCD_OK;
  }
  launch_pack_spinor(G, kFP64, R.n, R.w.b64, (const double*)R.b_dev, 1.0, 0, R.w.partials, st);
  launch_outer_residual_norm(R.n, R.w.sc, R.w.partials, site_grid(G), p->s, st);
  HIP_TRY(hipMemcpyAsync(R.w.r64, R.w.b64, R.n * spinor_bytes(G, kFP64), hipMemcpyDeviceToDevice, st));
  launch_zero(G, kFP64, R.n, R.w.x64, st);
  if (dev) launch_ir_dev_start(R.n, R.w.sc, nullptr, p->tol, p->max_outer, st);
  return QCD_OK;
}

// The host's bookkeeping of a refinement before any scalar is read back.
void ir_init_host(IrRun& R) {
  for (int i = 0; i < R.n; i++) {
    R.outer[i] = R.inner_total[i] = 0;
    R.last_status[i] = kConverged;
    R.result[i] = QCD_OK;
    if (R.info) {
      R.info[i].history_len = 0;
      R.info[i].first_shat_over_s = 0;
      R.info[i].precond_steps = 0;
      R.info[i].precond_fallback = -1;
      R.info[i].precond_scale = 0;
    }
  }
  R.pc.net = R.net;
}

void ir_after_start(IrRun& R) {
  ir_init_host(R);
  R.any = false;
  for (int i = 0; i < R.n; i++) {
    const Scalars& h = R.g->host_sc[i];
    R.bn[i] = R.rn[i] = h.out_rnorm;
    if (!std::isfinite(R.bn[i])) R.result[i] = fail(QCD_ERR_ARG, "non-finite right-hand side %d", i);
    R.any |= h.outer_active && std::isfinite(R.bn[i]);
  }
  if (R.n == 1 && !std::isfinite(R.bn[0])) R.any = false;
}

// Even-odd: the refinement stops on the residual of the even system, whose
// norm equals that of b - D x after the odd half is reconstructed (its odd
// rows vanish), so the tolerance is taken relative to |b| rather than |b'|.
qcd_status ir_eo_scale_tol(IrRun& R, const qcd_ir_params* p, hipStream_t st) {
  qcd_gauge* g = const_cast<qcd_gauge*>(R.g);
  for (int i = 0; i < R.n; i++) {
    const double bp = g->host_sc[i].out_rnorm;
    if (bp > 0 && std::isfinite(bp)) g->host_sc[i].out_tol = p->tol * R.bfull[i] / bp;
    R.bn[i] = R.bfull[i];
  }
  HIP_TRY(hipMemcpyAsync(R.w.sc, g->host_sc, sizeof(Scalars) * R.n, hipMemcpyHostToDevice, st));
  return QCD_OK;
}

// y~ = low(r s/|r|), s^ = |single(y~)|, inner solver start (right-hand sides
// that met the tolerance are skipped by the kernels); x is saved first when a
// preconditioned step may have to be undone.
qcd_status ir_begin_step(IrRun& R, const qcd_ir_params* p, hipStream_t st) {
  const Geom G = R.w.eo ? half_geom(R.g->g) : R.g->g;  // geometry of the refined vectors
  const int prec = p->inner_prec;
  if (R.pc.net) HIP_TRY(hipMemcpyAsync(R.w.x64b, R.w.x64, R.n * spinor_bytes(G, kFP64), hipMemcpyDeviceToDevice, st));
  launch_convert(G, prec, R.n, R.w.sc, (const double*)R.w.r64, R.w.r, R.w.rstar, R.w.partials, p->inner.ftz, st);
  launch_convert_finish(R.n, R.w.sc, R.w.partials, site_grid(G), p->recalc_shat, p->s, st);
  HIP_LAUNCHED();
  if (R.pc.net && R.pc.scale == 0.0f) {  // c = 1 / gain of M, measured on the first y~
    double gain = 0;
    const void* y = R.w.r;
    if (R.w.eo) {  // the gain of M on (y~, 0)
      launch_copy_fields(G, kFP16, R.n, R.w.zin, spinor_elems(R.g->g), R.w.r, spinor_elems(G), st);
      y = R.w.zin;
    }
    qcd_status rc = ptc_gain(R.pc.net, R.n, y, &gain, st);
    if (rc) return rc;
    R.pc.scale = gain > 0 ? (float)(1.0 / gain) : 1.0f;
  }
  return QCD_OK;
}

// After the inner solve: bookkeeping, x += (|r| / s^) double(t~) (t~ = c M u~
// when preconditioned), r = b - D x in FP64 (skipped where not refining).
qcd_status ir_end_step(IrRun& R, const qcd_ir_params* p, hipStream_t st) {
  const Geom G = R.w.eo ? half_geom(R.g->g) : R.g->g;  // geometry of the refined vectors
  const int prec = p->inner_prec;
  memcpy(R.sc, R.g->host_sc, sizeof(Scalars) * R.n);
  for (int i = 0; i < R.n; i++) {
    R.inner_failed[i] = false;
    if (!R.sc[i].outer_active) continue;
    if (R.info && R.outer[i] == 0) R.info[i].first_shat_over_s = R.sc[i].shat / p->s;
    if (R.info && R.info[i].zeros && R.outer[i] < R.info[i].outer_history_cap)
      R.info[i].zeros[R.outer[i]] = R.sc[i].zeros;
    copy_history(R.info ? R.info + i : nullptr, R.w, i, R.sc[i].iter, R.sc[i].bnorm2, st);
    R.inner_total[i] += R.sc[i].iter;
    R.last_status[i] = R.sc[i].status;
    R.inner_failed[i] = R.sc[i].status == kNonFinite || R.sc[i].iter == 0;
    if (R.inner_failed[i] && !R.pc.net)
      R.result[i] = fail(R.sc[i].status == kNonFinite ? QCD_ERR_NONFINITE : QCD_ERR_BREAKDOWN,
                         "inner solve of right-hand side %d failed (status %d) in refinement step %d", i,
                         R.sc[i].status, R.outer[i]);
  }
  if (R.pc.net) {
    precond_apply(R.g, R.pc, R.w, R.n, R.w.x, R.w.z, p->inner.ftz, nullptr, st);
    launch_correct(G, prec, R.n, R.w.sc, (double*)R.w.x64, R.w.z, st);
  } else {
    launch_correct(G, prec, R.n, R.w.sc, (double*)R.w.x64, R.w.x, st);
  }
  residual64(R.g, R.kappa, R.w, nullptr, st);
  launch_outer_residual_norm(R.n, R.w.sc, R.w.partials, residual_rows(R.g, R.w), p->s, st);
  HIP_LAUNCHED();
  return QCD_OK;
}

// With the new residual norms in the host mirror: the flexible step is kept
// only if every refining residual dropped and stayed finite (else x is
// restored for the right-hand sides that failed and the run continues
// without the network); then the outer counters and stop flags.
qcd_status ir_after_step(IrRun& R, const qcd_ir_params* p, int step, hipStream_t st) {
  const Geom G = R.w.eo ? half_geom(R.g->g) : R.g->g;  // geometry of the refined vectors
  qcd_gauge* g = const_cast<qcd_gauge*>(R.g);
  if (R.pc.net) {
    bool undo = false;
    bool bad[kMaxRhs];
    for (int i = 0; i < R.n; i++) {
      bad[i] = false;
      if (!R.sc[i].outer_active) continue;
      const double r_new = g->host_sc[i].out_rnorm;
      bad[i] = R.inner_failed[i] || !std::isfinite(r_new) || !(r_new < R.rn[i]);
      undo |= bad[i];
    }
    if (undo) {
      for (int i = 0; i < R.n; i++)
        if (bad[i])
          HIP_TRY(hipMemcpyAsync((char*)R.w.x64 + i * spinor_bytes(G, kFP64),
                                 (char*)R.w.x64b + i * spinor_bytes(G, kFP64), spinor_bytes(G, kFP64),
                                 hipMemcpyDeviceToDevice, st));
      for (int i = 0; i < R.n; i++) g->host_sc[i].outer_active = R.sc[i].outer_active;
      HIP_TRY(hipMemcpyAsync(R.w.sc, g->host_sc, sizeof(Scalars) * R.n, hipMemcpyHostToDevice, st));
      residual64(R.g, R.kappa, R.w, nullptr, st);
      launch_outer_residual_norm(R.n, R.w.sc, R.w.partials, residual_rows(R.g, R.w), p->s, st);
      HIP_LAUNCHED();
      qcd_status rc = read_scalars(R.g, R.w, st);
      if (rc) return rc;
      R.pc_fallback = step;
      R.pc.net = nullptr;
    } else {
      R.pc_steps++;
    }
  }
  R.any = false;
  for (int i = 0; i < R.n; i++) {
    if (!R.sc[i].outer_active) continue;
    R.outer[i]++;
    R.rn[i] = g->host_sc[i].out_rnorm;
    if (R.info && R.info[i].outer_history && R.outer[i] - 1 < R.info[i].outer_history_cap)
      R.info[i].outer_history[R.outer[i] - 1] = R.rn[i] / R.bn[i];
    if (!std::isfinite(R.rn[i])) R.result[i] = fail(QCD_ERR_NONFINITE, "non-finite outer residual");
    if (R.result[i] < 0) {  // stop refining this right-hand side
      g->host_sc[i].outer_active = 0;
      HIP_TRY(hipMemcpyAsync(&R.w.sc[i].outer_active, &g->host_sc[i].outer_active, sizeof(int), hipMemcpyHostToDevice,
                             st));
    }
    R.any |= g->host_sc[i].outer_active != 0;
  }
  return QCD_OK;
}

qcd_status ir_finish(IrRun& R, double t0) {
  qcd_status res = QCD_OK;
  for (int i = 0; i < R.n; i++) {
    if (R.info) {
      qcd_solve_info& in = R.info[i];
      in.outer_iters = R.outer[i];
      in.inner_iters = R.inner_total[i];
      in.matvec_low = 2 * R.inner_total[i];
      in.matvec_fp64 = R.outer[i];
      in.true_rel_residual = R.bn[i] > 0 ? R.rn[i] / R.bn[i] : 0.0;
      in.inner_status = R.last_status[i];
      in.seconds = now_s() - t0;
      in.precond_steps = R.pc_steps;
      in.precond_fallback = R.pc_fallback;
      in.precond_scale = R.net ? R.pc.scale : 0.0;
    }
    res = worse(res, R.result[i]);
  }
  return res;
}

// The refinement with its steps run from the device: after the first step's
// conversion, each lattice is queued blocks of K inner iterations (replayed
// one-iteration graphs with use_graph, else direct launches) followed by one
// device step; a right-hand side whose inner solve stopped gets its
// correction, FP64 residual, stop test and next start in the first device
// step after it, and the kernels of everything else return at once.  The
// host polls after a number of blocks: K follows the inner iterations per
// refinement step seen so far (an iteration queued past an inner stop, or a
// device step queued before one, costs a few microseconds per launch), and
// the blocks per poll the steps that the residual reduction so far predicts
// to remain (a poll costs a host round trip with the GPU idle).  The first
// poll's K and blocks come from the handle's previous device-driven solve
// with the same tolerances and inner precision, else 4 and 2.  The host reads
// the device's step counts, stop reasons and log at the end.
qcd_status solve_ir_dev(IrRun* runs, int nrun, const qcd_ir_params* p, hipStream_t st) {
  qcd_status rc;
  std::vector<IrRun*> act;
  for (int r = 0; r < nrun; r++) {
    IrRun& R = runs[r];
    // the start (ir_start with dev) set the device's step bookkeeping; the host
    // mirror is refreshed at the first poll, until then every right-hand side counts as refining
    for (int i = 0; i < R.n; i++) R.g->host_sc[i].outer_active = 1;
    if ((rc = ir_begin_step(R, p, st))) return rc;  // the first conversion and inner start
    act.push_back(&R);
  }
  const int nact = (int)act.size();
  std::vector<hipGraphExec_t> gexec(nact, nullptr);
  std::vector<hipStream_t> rs(nact, st);
  std::vector<InnerRun> ir;
  const double hkey[4] = {p->tol, p->inner.tol, (double)p->inner_prec, (double)p->inner.even_odd};
  int K = 0, blocks = 0;
  for (int a = 0; a < nact; a++) {
    IrRun& R = *act[a];
    if (p->inner.use_graph &&
        (rc = iteration_graph(R.g, p->inner_prec, R.kappa, R.w, p->inner.ftz, Precond{}, &gexec[a])))
      return rc;
    if (nact > 1) rs[a] = R.g->cap_stream;
    ir.push_back(InnerRun{R.g, p->inner_prec, R.kappa, &R.w, Precond{}});
    if (!memcmp(R.g->hint_key, hkey, sizeof hkey)) {
      K = std::max(K, R.g->hint_iters);
      blocks = std::max(blocks, R.g->hint_steps);
    }
  }
  if (K <= 0 || blocks <= 0) {
    K = 4;
    blocks = 2;
  }
  // at most 256 iterations before the first poll: a call much easier than the
  // last one (a zero source after a hard solve) would otherwise queue many
  // blocks whose launches all return at once
  blocks = std::max(1, std::min(blocks, 256 / K));
  auto refining = [](const IrRun& R) {
    for (int i = 0; i < R.n; i++)
      if (R.g->host_sc[i].outer_active) return true;
    return false;
  };
  long launched = 0;
  const long cap = (long)p->max_outer * ((long)p->inner.max_iter + 2) + 8;
  while (nact > 0) {
    bool any = false;
    if (nact > 1) HIP_TRY(hipEventRecord(act[0]->g->ev_fork, st));
    for (int a = 0; a < nact; a++) {
      IrRun& R = *act[a];
      if (!refining(R)) continue;
      any = true;
      if (nact > 1) HIP_TRY(hipStreamWaitEvent(rs[a], act[0]->g->ev_fork, 0));
      for (int b = 0; b < blocks; b++) {
        for (int j = 0; j < K; j++) {
          if (gexec[a])
            HIP_TRY(hipGraphLaunch(gexec[a], rs[a]));
          else
            bicg_iteration(R.g, p->inner_prec, R.kappa, R.w, p->inner.ftz, Precond{}, rs[a]);
        }
        device_step(R.g, R.kappa, R.w, p, rs[a]);
      }
      if (nact > 1) {
        HIP_TRY(hipEventRecord(R.g->ev_done, rs[a]));
        HIP_TRY(hipStreamWaitEvent(st, R.g->ev_done, 0));
      }
    }
    if (!any) break;
    HIP_LAUNCHED();
    launched += (long)blocks * K;
    if ((rc = read_scalars_all(ir.data(), nact, st))) return rc;
    if (launched > cap) break;
    int kn = 1, rem = 1;
    for (int a = 0; a < nact; a++)
      for (int i = 0; i < act[a]->n; i++) {
        const Scalars& h = act[a]->g->host_sc[i];
        if (!h.outer_active) continue;
        if (h.outer_count > 0) {
          kn = std::max(kn, (h.inner_total + h.outer_count - 1) / h.outer_count);
          // steps still needed at the mean reduction per step so far
          const double rel = h.out_rnorm / h.out_bnorm, goal = h.out_tol;
          const double rate = std::pow(rel, 1.0 / h.outer_count);
          int need = 2;
          if (rel > goal && rate > 0.0 && rate < 0.999)
            need = (int)std::min(64.0, std::max(1.0, std::ceil(std::log(goal / rel) / std::log(rate))));
          rem = std::max(rem, need);
        } else {
          kn = std::max(kn, h.iter + 1);  // the first inner solve runs on
          rem = std::max(rem, 2);
        }
      }
    K = std::min(64, kn);
    blocks = rem;
  }
  // the hint for the next device-driven solve on each handle
  for (int a = 0; a < nact; a++) {
    IrRun& R = *act[a];
    qcd_gauge* g = const_cast<qcd_gauge*>(R.g);
    int it = 0, st_max = 0;
    for (int i = 0; i < R.n; i++) {
      const Scalars& h = g->host_sc[i];
      if (h.outer_count <= 0) continue;
      st_max = std::max(st_max, h.outer_count);
      it = std::max(it, (h.inner_total + h.outer_count - 1) / h.outer_count);
    }
    g->hint_iters = std::min(64, it);
    g->hint_steps = std::min(64, st_max);
    memcpy(g->hint_key, hkey, sizeof hkey);
  }
  // the device's bookkeeping: counts, stop reasons and the last |r| from the
  // scalars of the last poll; the step log is copied into the handle's pinned
  // buffer behind the work still to come and read after the final synchronisation
  for (int a = 0; a < nact; a++) {
    IrRun& R = *act[a];
    HIP_TRY(hipMemcpyAsync(R.g->host_log, R.w.outer_log, sizeof(double) * 2 * kOuterLog * R.n,
                           hipMemcpyDeviceToHost, st));
    R.log_pending = true;
    for (int i = 0; i < R.n; i++) {
      const Scalars& h = R.g->host_sc[i];
      R.bn[i] = h.bfull;
      R.rn[i] = h.out_rnorm;
      if (!std::isfinite(R.bn[i])) R.result[i] = fail(QCD_ERR_ARG, "non-finite right-hand side %d", i);
      R.outer[i] = h.outer_count;
      R.inner_total[i] = h.inner_total;
      R.last_status[i] = h.last_status;
      if (h.fail)
        R.result[i] = fail(h.fail == kNonFinite ? QCD_ERR_NONFINITE : QCD_ERR_BREAKDOWN,
                           "inner solve of right-hand side %d failed (status %d) in refinement step %d", i,
                           h.last_status, h.outer_count - 1);
      else if (h.outer_active || (h.outer_count > 0 && h.out_rnorm > h.out_tol * h.out_bnorm))
        R.result[i] = worse(R.result[i], QCD_NOT_CONVERGED);
      if (R.info) R.info[i].first_shat_over_s = h.outer_count > 0 ? h.first_shat / p->s : 0.0;
    }
  }
  return QCD_OK;
}

// The per-step residuals and zero counts of a device-driven refinement, from
// the handle's pinned copy of the step log (after the stream has synchronised).
void dev_log_to_info(IrRun& R) {
  if (!R.log_pending) return;
  R.log_pending = false;
  if (!R.info) return;
  const double* log = R.g->host_log;
  for (int i = 0; i < R.n; i++) {
    qcd_solve_info& in = R.info[i];
    for (int k = 0; k < R.outer[i] && k < kOuterLog; k++) {
      if (in.outer_history && k < in.outer_history_cap)
        in.outer_history[k] = log[((size_t)i * kOuterLog + k) * 2] / R.bn[i];
      if (in.zeros && k < in.outer_history_cap) in.zeros[k] = log[((size_t)i * kOuterLog + k) * 2 + 1];
    }
  }
}

// The refinement of Alg. 3 for several lattices at once: every refinement
// step converts all of them, runs their inner solves together
// (bicg_loop_multi) and corrects them.  runs[r].w must be set.
qcd_status solve_ir_runs(IrRun* runs, int nrun, const qcd_ir_params* p, hipStream_t st, double t0) {
  qcd_status rc;
  // the steps run from the device unless the host is asked to poll every
  // check_every iterations, or a network (whose step may be undone from the
  // host), per-step inner histories or more steps than the device log holds
  // are asked for
  bool dev = p->inner.check_every <= 0 && p->max_outer <= kOuterLog;
  for (int r = 0; r < nrun; r++) {
    if (runs[r].net) dev = false;
    if (runs[r].info)
      for (int i = 0; i < runs[r].n; i++)
        if (runs[r].info[i].history && runs[r].info[i].history_cap > 0) dev = false;
  }
  for (int r = 0; r < nrun; r++)
    if ((rc = ir_start(runs[r], p, st, dev))) return rc;
  HIP_LAUNCHED();
  if (dev) {
    for (int r = 0; r < nrun; r++) ir_init_host(runs[r]);
    if ((rc = solve_ir_dev(runs, nrun, p, st))) return rc;
  } else {
    std::vector<InnerRun> ir(nrun);
    for (int r = 0; r < nrun; r++) ir[r] = InnerRun{runs[r].g, p->inner_prec, runs[r].kappa, &runs[r].w, Precond{}};
    if ((rc = read_scalars_all(ir.data(), nrun, st))) return rc;
    for (int r = 0; r < nrun; r++) {
      runs[r].pc.scale = (float)p->precond_scale;
      ir_after_start(runs[r]);
      if (runs[r].w.eo && (rc = ir_eo_scale_tol(runs[r], p, st))) return rc;
    }
  }
  for (int step = 0; !dev; step++) {
    std::vector<IrRun*> act;
    for (int r = 0; r < nrun; r++)
      if (runs[r].any) act.push_back(&runs[r]);
    if (act.empty()) break;
    if (step >= p->max_outer) {
      for (IrRun* R : act)
        for (int i = 0; i < R->n; i++)
          if (R->g->host_sc[i].outer_active) R->result[i] = worse(R->result[i], QCD_NOT_CONVERGED);
      break;
    }
    for (IrRun* R : act)
      if ((rc = ir_begin_step(*R, p, st))) return rc;
    std::vector<InnerRun> ir;
    for (IrRun* R : act) ir.push_back(InnerRun{R->g, p->inner_prec, R->kappa, &R->w, R->pc});
    if ((rc = bicg_loop_multi(ir.data(), (int)ir.size(), p->inner, st, false))) return rc;
    for (IrRun* R : act)
      if ((rc = ir_end_step(*R, p, st))) return rc;
    if ((rc = read_scalars_all(ir.data(), (int)ir.size(), st))) return rc;
    for (IrRun* R : act)
      if ((rc = ir_after_step(*R, p, step, st))) return rc;
  }
  for (int r = 0; r < nrun; r++) {
    IrRun& R = runs[r];
    if (R.w.eo) {
      // x_o from x_e, the canonical solution, and |b - D x| of the full system for the report
      // The even rows of b - D x are those of the last refinement step's FP64
      // residual eta_e + kappa H_eo eta_o - (x_e - kappa^2 H_eo H_oe x_e), taken
      // at the x_e returned (the two forms agree in exact arithmetic; here they
      // differ by the rounding of the stored x_o), so only the odd rows are
      // computed again, in the reconstruction launch.  A network run may have
      // undone its last step, so there the even rows are recomputed.
      // Without a network the last step's residual also left H_oe x_e of the
      // returned x_e in t64 (every right-hand side took a step; else x_e = 0
      // never met that launch), so x_o = eta_o + kappa t64 needs no hop.
      double r2[kMaxRhs];
      const bool even_rows = R.net != nullptr;
      bool hop_kept = !even_rows;
      for (int i = 0; i < R.n; i++) hop_kept = hop_kept && R.outer[i] > 0;
      if ((rc = eo_finish(R.g, R.kappa, R.w, R.x_dev, r2, st, even_rows, hop_kept))) return rc;
      for (int i = 0; i < R.n; i++)
        if (R.outer[i] > 0) R.rn[i] = sqrt(r2[i] + (even_rows ? 0.0 : R.rn[i] * R.rn[i]));
    } else {
      launch_unpack_spinor(R.g->g, kFP64, R.n, (double*)R.x_dev, R.w.x64, nullptr, 1.0, st);
    }
  }
  HIP_LAUNCHED();
  HIP_TRY(hipStreamSynchronize(st));
  qcd_status res = QCD_OK;
  for (int r = 0; r < nrun; r++) {
    dev_log_to_info(runs[r]);
    res = worse(res, ir_finish(runs[r], t0));
  }
  return res;
}

// Workspace of qcd_solve_mixed_ir_static: a fixed device array of the library,
// one instance per GPU (each device holds it at its own address from module
// load to process end).  Host code uses the address hipGetSymbolAddress
// returns for the current device, never the array's name.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The current device's address of `scratch`, looked up once per device.
qcd_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(QCD_ERR_UNSUPPORTED, "device %d is beyond the %d devices the static workspace serves", dev,
                kScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(QCD_ERR_HIP, "hipGetSymbolAddress of the static workspace: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return QCD_OK;
}

qcd_status check_ir_params(const qcd_ir_params* p) {
  if (!p) return fail(QCD_ERR_ARG, "null parameters");
  if (!(p->tol > 0) || p->max_outer <= 0 || !(p->s > 0)) return fail(QCD_ERR_ARG, "tol > 0, max_outer > 0, s > 0 required");
  return check_bicg_params(&p->inner);
}

}  // namespace

extern "C" {

qcd_status qcd_solve_mixed_ir(const qcd_gauge* g, double kappa, int nrhs, void* x_dev, const void* b_dev,
                              const qcd_ir_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const double t0 = now_s();
  qcd_status rc = check_ir_params(p);
  if (rc) return rc;
  IrRun R;
  R.g = g;
  R.kappa = kappa;
  R.n = nrhs;
  R.x_dev = x_dev;
  R.b_dev = b_dev;
  R.info = info;
  R.net = const_cast<qcd_ptc*>(p->precond);
  if ((rc = check_ir_run(R, p))) return rc;
  const int what = (R.net ? 3 : 0) | (p->inner.even_odd ? kWhatEO : 0);
  if ((rc = get_work(g, what, p->inner_prec, p->inner.max_iter, nrhs, ws, ws_bytes, &R.w))) return rc;
  return solve_ir_runs(&R, 1, p, S(stream), t0);
}

qcd_status qcd_solve_mixed_ir_static(const qcd_gauge* g, double kappa, int nrhs, void* x_dev, const void* b_dev,
                                     const qcd_ir_params* p, qcd_solve_info* info, void* stream) {
  const double t0 = now_s();
  qcd_status rc = check_ir_params(p);
  if (rc) return rc;
  if (p->precond) return fail(QCD_ERR_UNSUPPORTED, "the static-workspace solve takes no network preconditioner");
  if (p->inner.use_graph)
    return fail(QCD_ERR_UNSUPPORTED, "the static-workspace solve does not capture graphs (instantiation allocates)");
  IrRun R;
  R.g = g;
  R.kappa = kappa;
  R.n = nrhs;
  R.x_dev = x_dev;
  R.b_dev = b_dev;
  R.info = info;
  if ((rc = check_ir_run(R, p))) return rc;
  const int what = p->inner.even_odd ? kWhatEO : 0;
  const size_t need = carve(g, what, p->inner_prec, p->inner.max_iter, nrhs, nullptr).bytes;
  if (need > kScratchBytes)
    return fail(QCD_ERR_WORKSPACE, "the solve needs %zu bytes of workspace; the static workspace holds %zu", need,
                kScratchBytes);
  void* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  if ((rc = get_work(g, what, p->inner_prec, p->inner.max_iter, nrhs, base, kScratchBytes, &R.w))) return rc;
  return solve_ir_runs(&R, 1, p, S(stream), t0);
}

qcd_status qcd_solve_mixed_ir_batched(int nlat, const qcd_gauge* const* g, const double* kappa, const int* nrhs,
                                      void* const* x_dev, const void* const* b_dev, const qcd_ir_params* p,
                                      qcd_solve_info* const* info, void* const* ws, const size_t* ws_bytes,
                                      void* stream) {
  const double t0 = now_s();
  qcd_status rc = check_ir_params(p);
  if (rc) return rc;
  if (nlat < 1 || nlat > 64 || !g || !kappa || !nrhs || !x_dev || !b_dev)
    return fail(QCD_ERR_ARG, "nlat must be in 1..64 and the arrays non-null");
  if (p->precond) return fail(QCD_ERR_UNSUPPORTED, "a network preconditioner serves one lattice; use qcd_solve_mixed_ir");
  std::vector<IrRun> runs(nlat);
  for (int r = 0; r < nlat; r++) {
    for (int q = 0; q < r; q++)
      if (g[q] == g[r]) return fail(QCD_ERR_ARG, "lattice %d repeats the gauge handle of lattice %d", r, q);
    IrRun& R = runs[r];
    R.g = g[r];
    R.kappa = kappa[r];
    R.n = nrhs[r];
    R.x_dev = x_dev[r];
    R.b_dev = b_dev[r];
    R.info = info ? info[r] : nullptr;
    if ((rc = check_ir_run(R, p))) return rc;
    void* wr = ws ? ws[r] : nullptr;
    const size_t wb = (ws && ws_bytes) ? ws_bytes[r] : 0;
    if ((rc = get_work(g[r], p->inner.even_odd ? kWhatEO : 0, p->inner_prec, p->inner.max_iter, nrhs[r], wr, wb,
                       &R.w)))
      return rc;
  }
  return solve_ir_runs(runs.data(), nlat, p, S(stream), t0);
}


qcd_status qcd_stream_probe(void* dst_dev, const void* src_dev, size_t bytes, int mode, int reps, double* us,
                            void* stream) {
  if (!us || mode < 0 || mode > 2 || reps < 1 || reps > 10000 || bytes == 0 || bytes % 16)
    return fail(QCD_ERR_ARG, "mode 0..2, reps 1..10000, bytes a positive multiple of 16 and an output are required");
  if (!dst_dev || (mode < 2 && !src_dev)) return fail(QCD_ERR_ARG, "null buffer");
  hipStream_t st = S(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(QCD_ERR_HIP, "hipEventCreate failed");
  }
  launch_stream_probe(mode, dst_dev, src_dev, bytes, st);  // warm-up
  (void)hipEventRecord(e0, st);
  for (int i = 0; i < reps; i++) launch_stream_probe(mode, dst_dev, src_dev, bytes, st);
  (void)hipEventRecord(e1, st);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(QCD_ERR_HIP, "probe timing: %s", hipGetErrorString(e));
  HIP_LAUNCHED();
  *us = (double)ms * 1e3 / reps;
  return QCD_OK;
}

// ---------------------------------------------------------------------------
// Extreme |eigenvalues| of the even-odd matrix (a diagnostic).

}  // extern "C"

namespace {

// logs[k] = log of sqrt(sums[num] / sums[den]) (den < 0: / 1), scale = 1 / sqrt(sums[num])
__global__ void k_log_ratio(const double* __restrict__ sums, int num, int den, double* __restrict__ logs, int k,
                            double* __restrict__ scale) {
  if (threadIdx.x != 0) return;
  const double a = sums[num], b = den >= 0 ? sums[den] : 1.0;
  if (logs) logs[k] = 0.5 * log(a / b);
  scale[0] = 1.0 / sqrt(a);
}

struct SpecBufs {
  void* p[8] = {};
  ~SpecBufs() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
};

// x = y / |y| for an even-parity FP64 field y (x != y), and log |y| / |x_prev|
// (|x_prev| = 1) into logs[k] if logs is not null.
void spec_normalise(const Geom& gh, double* x, const double* y, double* partials, double* sums, double* scale,
                    double* logs, int k, hipStream_t st) {
  launch_narrow(gh, kFP64, 1, x, y, partials, 0, st);  // a copy; the partials hold |y|^2
  launch_finish_sum(1, partials, site_grid(gh), 1, sums, st);
  hipLaunchKernelGGL(k_log_ratio, dim3(1), dim3(64), 0, st, sums, 0, -1, logs, k, scale);
  launch_widen(gh, kFP64, 1, x, y, scale, st);
}

// x = v / |v| for the even half v of a seeded Gaussian field.
void spec_start(const qcd_gauge* g, uint64_t seed, double* xe, double* tmp, double* to, double* canon,
                double* partials, double* sums, double* scale, hipStream_t st) {
  const Geom& G = g->g;
  launch_gaussian(canon, (int64_t)2 * G.Vh * 12, seed, st);
  launch_pack_spinor_split(G, 1, tmp, to, canon, nullptr, st);
  spec_normalise(half_geom(G), xe, tmp, partials, sums, scale, nullptr, 0, st);
}

double mean_tail(const std::vector<double>& v, int from, int to) {
  double s = 0;
  for (int k = from; k < to; k++) s += v[k];
  return s / (to - from);
}

}  // namespace

extern "C" {

qcd_status qcd_eo_spectrum(const qcd_gauge* g, double kappa, int power_iters, int inverse_iters, uint64_t seed,
                           double* abs_max, double* abs_min, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if (!abs_max || !abs_min) return fail(QCD_ERR_ARG, "null output");
  if (!(kappa > 0) || !std::isfinite(kappa)) return fail(QCD_ERR_ARG, "kappa must be positive and finite");
  if (power_iters < 2 || power_iters > 100000 || inverse_iters < 0 || inverse_iters > 1000)
    return fail(QCD_ERR_ARG, "power_iters must be in 2..100000 and inverse_iters in 0..1000");
  hipStream_t st = S(stream);
  const Geom& G = g->g;
  const Geom gh = half_geom(G);
  const DslashTune& tu = g->tune[kFP64];
  const int erows = dslash_partial_rows(G, tu, 1, true);
  const int nrows = std::max(erows, site_grid(gh));
  const int nlog = power_iters + inverse_iters;
  const size_t sizes[8] = {spinor_bytes(gh, kFP64), spinor_bytes(gh, kFP64), spinor_bytes(gh, kFP64),
                           canon_bytes(G), canon_bytes(G), (size_t)nrows * 4 * sizeof(double),
                           8 * sizeof(double), (size_t)nlog * sizeof(double)};
  SpecBufs B;
  for (int i = 0; i < 8; i++) HIP_TRY(hipMalloc(&B.p[i], sizes[i]));
  double *xe = (double*)B.p[0], *ye = (double*)B.p[1], *to = (double*)B.p[2];
  double *cb = (double*)B.p[3], *cx = (double*)B.p[4], *partials = (double*)B.p[5];
  double *sums = (double*)B.p[6], *scale = sums + 4, *logs = (double*)B.p[7];
  const void* U = g->U[kFP64];
  const double k2 = kappa * kappa;
  // power iteration: y = A x, log |y| / |x| recorded, x = y / |y|
  spec_start(g, seed, xe, ye, to, cx, partials, sums, scale, st);
  for (int k = 0; k < power_iters; k++) {
    launch_dslash(kFP64, G, tu, kOpH, kEpiNone, 1, to, xe, U, 1.0, nullptr, nullptr, nullptr, 0, st, nullptr, 1);
    launch_dslash(kFP64, G, tu, kOpD, kEpiTS, 1, ye, to, U, k2, nullptr, partials, nullptr, 0, st, xe, 0);
    launch_finish_sum(1, partials, erows, 4, sums, st);
    hipLaunchKernelGGL(k_log_ratio, dim3(1), dim3(64), 0, st, sums, 2, 3, logs, k, scale);
    launch_widen(gh, kFP64, 1, xe, ye, scale, st);
  }
  HIP_LAUNCHED();
  // inverse iteration: A^-1 x is the even half of D^-1 (x, 0) (eq. (5) with b_o = 0)
  if (inverse_iters > 0) {
    qcd_ir_params p{};
    p.tol = 1e-12;
    p.max_outer = 100;
    p.inner_prec = g->U[kFP16] ? QCD_FP16 : QCD_FP64;
    p.s = 128.0;
    p.recalc_shat = 1;
    p.inner.tol = 1e-2;
    p.inner.max_iter = 10000;
    p.inner.sigma = 64.0;
    p.inner.recalc_gamma = 1;
    p.inner.omega0 = 0.7;
    p.inner.even_odd = 1;
    spec_start(g, seed + 1, xe, ye, to, cx, partials, sums, scale, st);
    for (int k = 0; k < inverse_iters; k++) {
      launch_zero(gh, kFP64, 1, to, st);
      launch_unpack_spinor_split(G, 1, cb, xe, to, st);
      HIP_LAUNCHED();
      qcd_solve_info info{};
      rc = qcd_solve_mixed_ir(g, kappa, 1, cx, cb, &p, &info, nullptr, 0, stream);
      if (rc != QCD_OK) return rc == QCD_NOT_CONVERGED ? fail(rc, "an inverse-iteration solve did not converge") : rc;
      launch_pack_spinor_split(G, 1, ye, to, cx, nullptr, st);
      spec_normalise(gh, xe, ye, partials, sums, scale, logs, power_iters + k, st);
      HIP_LAUNCHED();
    }
  }
  std::vector<double> h(nlog);
  HIP_TRY(hipMemcpyAsync(h.data(), logs, nlog * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *abs_max = std::exp(mean_tail(h, power_iters / 2, power_iters));
  *abs_min = inverse_iters > 0 ? std::exp(-mean_tail(h, power_iters + inverse_iters / 2, nlog)) : NAN;
  if (!std::isfinite(*abs_max) || (inverse_iters > 0 && !std::isfinite(*abs_min)))
    return fail(QCD_ERR_NONFINITE, "the spectrum estimate is not finite");
  return QCD_OK;
}

}  // extern "C"
