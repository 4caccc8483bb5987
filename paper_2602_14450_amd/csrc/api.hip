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
#include <string>

#include "qcd.h"
#include "internal.h"

using namespace qcd;

struct qcd_gauge {
  Geom g;
  int dims[4];
  void* U[3];
  void* ws;          // cached workspace used when the caller passes none
  size_t ws_bytes;
  Scalars* host_sc;  // pinned mirror of the device scalars
  DslashTune tune[3];
};

namespace {

thread_local std::string g_err;

qcd_status fail(qcd_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
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

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t spinor_bytes(const Geom& g, int prec) { return spinor_elems(g) * prec_complex_bytes(prec); }
size_t partial_bytes(const Geom& g) {
  int rows = site_grid(g);
  for (int p = 0; p < 3; p++) rows = std::max(rows, flat_rows(g, p));
  rows = std::max(rows, dslash_partial_rows(g));
  return (size_t)rows * 8 * sizeof(double);
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
  double2* x64 = nullptr;
  double2* b64 = nullptr;
  double2* r64 = nullptr;
  void* x = nullptr;
  void* r = nullptr;
  void* rstar = nullptr;
  void* p = nullptr;
  void* v = nullptr;
  void* t = nullptr;
  double* partials = nullptr;
  Scalars* sc = nullptr;
  double* history = nullptr;
  double* sums = nullptr;
  size_t bytes = 0;
};

// what: 0 refinement, 1 BiCGStab, 2 operator with canonical layout
Work carve(const Geom& g, int what, int prec, int max_iter, char* base) {
  Carve c{base};
  Work w;
  if (what == 0 || what == 1) {
    w.x64 = (double2*)c.take(spinor_bytes(g, kFP64));
    w.b64 = (double2*)c.take(spinor_bytes(g, kFP64));
    w.r64 = (double2*)c.take(spinor_bytes(g, kFP64));
    w.x = c.take(spinor_bytes(g, prec));
    w.r = c.take(spinor_bytes(g, prec));
    w.rstar = c.take(spinor_bytes(g, prec));
    w.p = c.take(spinor_bytes(g, prec));
    w.v = c.take(spinor_bytes(g, prec));
    w.t = c.take(spinor_bytes(g, prec));
    w.history = (double*)c.take(sizeof(double) * (size_t)(max_iter > 0 ? max_iter : 1));
  } else {
    w.x = c.take(spinor_bytes(g, prec));
    w.r = c.take(spinor_bytes(g, prec));
  }
  w.partials = (double*)c.take(partial_bytes(g));
  w.sc = (Scalars*)c.take(sizeof(Scalars));
  w.sums = (double*)c.take(8 * sizeof(double));
  w.bytes = c.off;
  return w;
}

qcd_status get_work(const qcd_gauge* gc, int what, int prec, int max_iter, void* ws, size_t ws_bytes, Work* out) {
  qcd_gauge* g = const_cast<qcd_gauge*>(gc);
  Work need = carve(g->g, what, prec, max_iter, nullptr);
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
  *out = carve(g->g, what, prec, max_iter, base);
  return QCD_OK;
}

bool valid_prec(int p) { return p == kFP64 || p == kFP32 || p == kFP16; }

qcd_status check_gauge(const qcd_gauge* g, int prec) {
  if (!g) return fail(QCD_ERR_ARG, "null gauge handle");
  if (!valid_prec(prec)) return fail(QCD_ERR_ARG, "invalid precision %d", prec);
  if (!g->U[prec]) return fail(QCD_ERR_ARG, "gauge handle holds no links in precision %d", prec);
  return QCD_OK;
}

qcd_status read_scalars(const qcd_gauge* g, const Work& w, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(g->host_sc, w.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return QCD_OK;
}

qcd_status read_sum(const Work& w, int nrows, int nv, double* out, hipStream_t st) {
  launch_finish_sum(w.partials, nrows, nv, w.sums, st);
  HIP_LAUNCHED();
  HIP_TRY(hipMemcpyAsync(out, w.sums, nv * sizeof(double), hipMemcpyDeviceToHost, st));
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
}

qcd_status check_bicg_params(const qcd_bicgstab_params* p) {
  if (!p) return fail(QCD_ERR_ARG, "null parameters");
  if (!(p->tol >= 0) || p->max_iter <= 0) return fail(QCD_ERR_ARG, "tol must be >= 0 and max_iter > 0");
  if (p->sigma < 0 || p->sigma_lambda < 0 || p->omega0 < 0 || p->omega0 > 1)
    return fail(QCD_ERR_ARG, "sigma, sigma_lambda >= 0 and 0 <= omega0 <= 1 required");
  return QCD_OK;
}

// One BiCGStab iteration of Alg. 4 / Alg. 5, entirely on the device.
void bicg_iteration(const qcd_gauge* g, int prec, double kappa, const Work& w, int ftz, hipStream_t st) {
  const Geom& G = g->g;
  const int drows = dslash_partial_rows(G), frows = flat_rows(G, prec);
  const void* U = g->U[prec];
  const DslashTune& tu = g->tune[prec];
  launch_p_update(G, prec, w.sc, w.p, w.v, w.r, ftz, st);
  launch_dslash(prec, G, tu, kOpD, kEpiDotAux, w.v, w.p, U, kappa, w.rstar, w.partials, &w.sc->active, ftz, st);
  launch_alpha(w.sc, w.partials, drows, st);
  launch_s_update(G, prec, w.sc, w.r, w.v, ftz, st);
  launch_dslash(prec, G, tu, kOpD, kEpiTS, w.t, w.r, U, kappa, nullptr, w.partials, &w.sc->active, ftz, st);
  launch_omega(w.sc, w.partials, drows, st);
  launch_xr_update(G, prec, w.sc, w.x, w.r, w.t, w.p, w.rstar, w.partials, ftz, st);
  launch_iter_end(w.sc, w.partials, frows, w.history, st);
}

// FP64 residual r = b - D x with |r|^2 partials (one row per Wilson-operator block).
void residual64(const qcd_gauge* g, double kappa, const Work& w, hipStream_t st) {
  launch_dslash(kFP64, g->g, g->tune[kFP64], kOpD, kEpiResid, w.r64, w.x64, g->U[kFP64], kappa, w.b64, w.partials,
                nullptr, 0, st);
}

// Run the inner loop from initialised scalars until the device reports a
// stop; fills the host mirror.  Iterations are queued in chunks without host
// synchronisation (kernels of a stopped solve return at once).  After the
// first chunk, the chunk length is the number of iterations the observed
// convergence rate predicts are still needed, plus one.
qcd_status bicg_loop(const qcd_gauge* g, int prec, double kappa, const Work& w, const qcd_bicgstab_params& p,
                     hipStream_t st) {
  const int K0 = p.check_every > 0 ? p.check_every : 4;
  qcd_status s = read_scalars(g, w, st);
  if (s) return s;
  int launched = 0, chunk = K0;
  double prev_res2 = g->host_sc->bnorm2;
  int prev_iter = 0;
  while (g->host_sc->active && launched <= p.max_iter + K0) {
    for (int j = 0; j < chunk; j++) bicg_iteration(g, prec, kappa, w, p.ftz, st);
    HIP_LAUNCHED();
    launched += chunk;
    s = read_scalars(g, w, st);
    if (s) return s;
    const Scalars& h = *g->host_sc;
    if (!h.active) break;
    chunk = K0;
    if (p.check_every <= 0 && h.iter > prev_iter) {
      const double res2 = h.rnorm2 / (h.gamma_cum * h.gamma_cum);
      const double target = h.tol2 * h.bnorm2;
      const double rate = std::pow(res2 / prev_res2, 1.0 / (h.iter - prev_iter));  // per iteration
      if (rate > 0.0 && rate < 0.999 && res2 > target) {
        const double need = std::log(target / res2) / std::log(rate);
        chunk = (int)std::min(64.0, std::max(1.0, std::ceil(need) + 1.0));
      }
      prev_res2 = res2;
      prev_iter = h.iter;
    }
  }
  return QCD_OK;
}

void copy_history(qcd_solve_info* info, const Work& w, int n, double bn2, hipStream_t st) {
  if (!info || !info->history || info->history_cap <= info->history_len || n <= 0) return;
  int m = n;
  if (m > info->history_cap - info->history_len) m = info->history_cap - info->history_len;
  if (hipMemcpyAsync(info->history + info->history_len, w.history, m * sizeof(double), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
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
  if (prec_mask == 0) prec_mask = 7;
  prec_mask |= 1 << kFP64;
  qcd_gauge* g = new qcd_gauge();
  memset(g, 0, sizeof(*g));
  g->g = make_geom(dims);
  // defaults measured on MI355X at 32^3 x 64 (the tuner may override them)
  g->tune[kFP64] = DslashTune{1, 0};
  g->tune[kFP32] = DslashTune{1, 1};
  g->tune[kFP16] = DslashTune{1, 1};
  memcpy(g->dims, dims, sizeof g->dims);
  hipStream_t st = S(stream);
  qcd_status rc = QCD_OK;
  for (int p = 0; p < 3 && rc == QCD_OK; p++) {
    if (!(prec_mask & (1 << p))) continue;
    size_t bytes = link_elems(g->g) * prec_complex_bytes(p);
    if (hipMalloc(&g->U[p], bytes) != hipSuccess) {
      g->U[p] = nullptr;
      rc = fail(QCD_ERR_HIP, "hipMalloc of %zu bytes for links failed", bytes);
      break;
    }
    // the padding of the last 64-site block stays zero
    if (hipMemsetAsync(g->U[p], 0, bytes, st) != hipSuccess) rc = fail(QCD_ERR_HIP, "hipMemsetAsync failed");
    launch_pack_links(g->g, p, g->U[p], (const double*)U_dev, st);
    if (hipGetLastError() != hipSuccess) rc = fail(QCD_ERR_HIP, "link packing launch failed");
  }
  if (rc == QCD_OK && hipHostMalloc((void**)&g->host_sc, sizeof(Scalars), 0) != hipSuccess)
    rc = fail(QCD_ERR_HIP, "hipHostMalloc failed");
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
  for (int p = 0; p < 3; p++)
    if (g->U[p]) (void)hipFree(g->U[p]);
  if (g->ws) (void)hipFree(g->ws);
  if (g->host_sc) (void)hipHostFree(g->host_sc);
  delete g;
  return QCD_OK;
}

qcd_status qcd_set_dslash_tuning(qcd_gauge* g, qcd_prec prec, int sched, int variant) {
  if (!g || !valid_prec(prec)) return fail(QCD_ERR_ARG, "invalid handle or precision");
  if (sched < 0 || sched > 1 || variant < 0 || variant >= kDslashVariants)
    return fail(QCD_ERR_ARG, "sched must be 0 or 1 and variant 0..%d", kDslashVariants - 1);
  g->tune[prec] = DslashTune{sched, variant};
  return QCD_OK;
}

qcd_status qcd_get_dslash_tuning(const qcd_gauge* g, qcd_prec prec, int* sched, int* variant) {
  if (!g || !valid_prec(prec) || !sched || !variant) return fail(QCD_ERR_ARG, "invalid argument");
  *sched = g->tune[prec].sched;
  *variant = g->tune[prec].variant;
  return QCD_OK;
}

size_t qcd_spinor_bytes(const qcd_gauge* g, qcd_prec prec) {
  if (!g || !valid_prec(prec)) return 0;
  return spinor_bytes(g->g, prec);
}

size_t qcd_workspace_bytes(const qcd_gauge* g, int what, qcd_prec prec, int max_iter) {
  if (!g || !valid_prec(prec) || what < 0 || what > 2) return 0;
  return carve(g->g, what, prec, max_iter, nullptr).bytes;
}

qcd_status qcd_convert(const qcd_gauge* g, qcd_prec prec, void* native_dev, const void* canonical_dev, double scale,
                       int ftz, double* norm2, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if (!valid_prec(prec) || !native_dev || !canonical_dev) return fail(QCD_ERR_ARG, "invalid argument");
  hipStream_t st = S(stream);
  Work w;
  if (norm2) {
    rc = get_work(g, 2, prec, 0, nullptr, 0, &w);
    if (rc) return rc;
  }
  launch_pack_spinor(g->g, prec, native_dev, (const double*)canonical_dev, scale, ftz, norm2 ? w.partials : nullptr,
                     st);
  HIP_LAUNCHED();
  if (norm2) return read_sum(w, site_grid(g->g), 1, norm2, st);
  return QCD_OK;
}

qcd_status qcd_unconvert(const qcd_gauge* g, qcd_prec prec, void* canonical_dev, const void* native_dev, double scale,
                         void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if (!valid_prec(prec) || !native_dev || !canonical_dev) return fail(QCD_ERR_ARG, "invalid argument");
  launch_unpack_spinor(g->g, prec, (double*)canonical_dev, native_dev, scale, S(stream));
  HIP_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_dslash(const qcd_gauge* g, double kappa, qcd_op op, qcd_prec prec, qcd_layout layout, void* out_dev,
                      const void* in_dev, void* stream) {
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if (!out_dev || !in_dev || out_dev == in_dev) return fail(QCD_ERR_ARG, "out and in must be distinct non-null buffers");
  if (op < QCD_OP_D || op > QCD_OP_HDAG) return fail(QCD_ERR_ARG, "invalid op %d", (int)op);
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  hipStream_t st = S(stream);
  if (layout == QCD_LAYOUT_NATIVE) {
    launch_dslash(prec, g->g, g->tune[prec], op, kEpiNone, out_dev, in_dev, g->U[prec], kappa, nullptr, nullptr,
                  nullptr, 0, st);
    HIP_LAUNCHED();
    return QCD_OK;
  }
  if (layout != QCD_LAYOUT_CANONICAL) return fail(QCD_ERR_ARG, "invalid layout");
  Work w;
  rc = get_work(g, 2, prec, 0, nullptr, 0, &w);
  if (rc) return rc;
  launch_pack_spinor(g->g, prec, w.x, (const double*)in_dev, 1.0, 0, nullptr, st);
  launch_dslash(prec, g->g, g->tune[prec], op, kEpiNone, w.r, w.x, g->U[prec], kappa, nullptr, nullptr, nullptr, 0,
                st);
  launch_unpack_spinor(g->g, prec, (double*)out_dev, w.r, 1.0, st);
  HIP_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_residual(const qcd_gauge* g, double kappa, void* r_dev, const void* x_dev, const void* b_dev,
                        double* norm2, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if (!r_dev || !x_dev || !b_dev) return fail(QCD_ERR_ARG, "null argument");
  hipStream_t st = S(stream);
  Work w;
  rc = get_work(g, 1, kFP64, 1, nullptr, 0, &w);
  if (rc) return rc;
  launch_pack_spinor(g->g, kFP64, w.x64, (const double*)x_dev, 1.0, 0, nullptr, st);
  launch_pack_spinor(g->g, kFP64, w.b64, (const double*)b_dev, 1.0, 0, nullptr, st);
  residual64(g, kappa, w, st);
  launch_unpack_spinor(g->g, kFP64, (double*)r_dev, w.r64, 1.0, st);
  HIP_LAUNCHED();
  if (norm2) return read_sum(w, dslash_partial_rows(g->g), 1, norm2, st);
  return QCD_OK;
}

qcd_status qcd_bicgstab(const qcd_gauge* g, double kappa, qcd_prec prec, void* x_dev, const void* b_dev,
                        const qcd_bicgstab_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const double t0 = now_s();
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if (!x_dev || !b_dev) return fail(QCD_ERR_ARG, "null vector");
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if ((rc = check_bicg_params(p))) return rc;
  hipStream_t st = S(stream);
  Work w;
  if ((rc = get_work(g, 1, prec, p->max_iter, ws, ws_bytes, &w))) return rc;
  const Geom& G = g->g;
  const int rows = site_grid(G);
  Scalars hs;
  init_params(&hs, *p);
  HIP_TRY(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, st));
  // r = r* = low(b), x0 = 0
  launch_pack_spinor(G, prec, w.r, (const double*)b_dev, 1.0, p->ftz, w.partials, st);
  HIP_TRY(hipMemcpyAsync(w.rstar, w.r, spinor_bytes(G, prec), hipMemcpyDeviceToDevice, st));
  launch_bicg_init(w.sc, w.partials, rows, st);
  HIP_LAUNCHED();
  if ((rc = bicg_loop(g, prec, kappa, w, *p, st))) return rc;
  const Scalars sc = *g->host_sc;
  const int iters = sc.iter;
  if (iters > 0) {
    launch_unpack_spinor(G, prec, (double*)x_dev, w.x, sc.xscale / sc.lambda_cum, st);
  } else {
    HIP_TRY(hipMemsetAsync(x_dev, 0, (size_t)G.Vh * 2 * 12 * 16, st));
  }
  HIP_LAUNCHED();
  // FP64 true residual of the returned solution
  double r2 = 0, b2 = 0;
  launch_pack_spinor(G, kFP64, w.b64, (const double*)b_dev, 1.0, 0, w.partials, st);
  if ((rc = read_sum(w, rows, 1, &b2, st))) return rc;
  launch_pack_spinor(G, kFP64, w.x64, (const double*)x_dev, 1.0, 0, nullptr, st);
  residual64(g, kappa, w, st);
  if ((rc = read_sum(w, dslash_partial_rows(G), 1, &r2, st))) return rc;
  if (info) {
    info->outer_iters = 0;
    info->inner_iters = iters;
    info->matvec_low = 2 * iters;
    info->matvec_fp64 = 1;
    info->true_rel_residual = b2 > 0 ? sqrt(r2 / b2) : 0.0;
    info->inner_status = sc.status;
    info->first_shat_over_s = 1.0;
    info->history_len = 0;
    copy_history(info, w, iters, sc.bnorm2, st);
    info->seconds = now_s() - t0;
  }
  switch (sc.status) {
    case kConverged: return QCD_OK;
    case kMaxIter: return QCD_NOT_CONVERGED;
    case kBreakdown: return fail(QCD_ERR_BREAKDOWN, "BiCGStab breakdown after %d iterations", iters);
    case kNonFinite: return fail(QCD_ERR_NONFINITE, "non-finite solver scalar after %d iterations", iters);
    default: return fail(QCD_ERR_HIP, "solver stopped in an unknown state %d", sc.status);
  }
}

qcd_status qcd_solve_mixed_ir(const qcd_gauge* g, double kappa, void* x_dev, const void* b_dev, const qcd_ir_params* p,
                              qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const double t0 = now_s();
  if (!p) return fail(QCD_ERR_ARG, "null parameters");
  qcd_status rc = check_gauge(g, p->inner_prec);
  if (rc) return rc;
  if (!x_dev || !b_dev) return fail(QCD_ERR_ARG, "null vector");
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if (!(p->tol > 0) || p->max_outer <= 0 || !(p->s > 0)) return fail(QCD_ERR_ARG, "tol > 0, max_outer > 0, s > 0 required");
  if ((rc = check_bicg_params(&p->inner))) return rc;
  const int prec = p->inner_prec;
  hipStream_t st = S(stream);
  Work w;
  if ((rc = get_work(g, 0, prec, p->inner.max_iter, ws, ws_bytes, &w))) return rc;
  const Geom& G = g->g;
  const int rows = site_grid(G);
  Scalars hs;
  init_params(&hs, p->inner);
  HIP_TRY(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, st));
  // b in the native FP64 layout; r = b, x = 0
  launch_pack_spinor(G, kFP64, w.b64, (const double*)b_dev, 1.0, 0, w.partials, st);
  launch_outer_residual_norm(w.sc, w.partials, rows, p->s, st);
  HIP_TRY(hipMemcpyAsync(w.r64, w.b64, spinor_bytes(G, kFP64), hipMemcpyDeviceToDevice, st));
  launch_zero(G, kFP64, w.x64, st);
  HIP_LAUNCHED();
  if ((rc = read_scalars(g, w, st))) return rc;
  const double bn = g->host_sc->out_rnorm;
  if (info) {
    info->history_len = 0;
    info->inner_iters = info->matvec_low = info->matvec_fp64 = info->outer_iters = 0;
    info->first_shat_over_s = 0;
  }
  int outer = 0, inner_total = 0, mv64 = 0, last_status = kConverged;
  qcd_status result = QCD_OK;
  double rn = bn;
  if (bn == 0.0 || !std::isfinite(bn)) {
    launch_zero(G, kFP64, w.x64, st);
    if (!std::isfinite(bn)) result = fail(QCD_ERR_ARG, "non-finite right-hand side");
    rn = bn;
  } else {
    while (true) {
      if (rn / bn <= p->tol) break;
      if (outer >= p->max_outer) { result = QCD_NOT_CONVERGED; break; }
      // y~ = low(r s/|r|), s^ = |single(y~)|, inner solver start
      launch_convert(G, prec, w.sc, (const double*)w.r64, w.r, w.rstar, w.x, w.partials, p->inner.ftz, st);
      launch_convert_finish(w.sc, w.partials, rows, p->recalc_shat, p->s, st);
      HIP_LAUNCHED();
      if ((rc = bicg_loop(g, prec, kappa, w, p->inner, st))) return rc;
      const Scalars sc = *g->host_sc;
      if (info && outer == 0) info->first_shat_over_s = sc.shat / p->s;
      if (info && info->zeros && outer < info->outer_history_cap) info->zeros[outer] = sc.zeros;
      copy_history(info, w, sc.iter, sc.bnorm2, st);
      inner_total += sc.iter;
      last_status = sc.status;
      if (sc.status == kNonFinite || sc.iter == 0) {
        // no usable correction from this step
        result = fail(sc.status == kNonFinite ? QCD_ERR_NONFINITE : QCD_ERR_BREAKDOWN,
                      "inner solve failed (status %d) in refinement step %d", sc.status, outer);
        break;
      }
      // x += (|r| / s^) double(t~); r = b - D x in FP64
      launch_correct(G, prec, w.sc, (double*)w.x64, w.x, st);
      residual64(g, kappa, w, st);
      launch_outer_residual_norm(w.sc, w.partials, dslash_partial_rows(G), p->s, st);
      HIP_LAUNCHED();
      mv64++;
      outer++;
      if ((rc = read_scalars(g, w, st))) return rc;
      rn = g->host_sc->out_rnorm;
      if (info && info->outer_history && outer - 1 < info->outer_history_cap) info->outer_history[outer - 1] = rn / bn;
      if (!std::isfinite(rn)) { result = fail(QCD_ERR_NONFINITE, "non-finite outer residual"); break; }
    }
  }
  launch_unpack_spinor(G, kFP64, (double*)x_dev, w.x64, 1.0, st);
  HIP_LAUNCHED();
  HIP_TRY(hipStreamSynchronize(st));
  if (info) {
    info->outer_iters = outer;
    info->inner_iters = inner_total;
    info->matvec_low = 2 * inner_total;
    info->matvec_fp64 = mv64;
    info->true_rel_residual = bn > 0 ? rn / bn : 0.0;
    info->inner_status = last_status;
    info->seconds = now_s() - t0;
  }
  return result;
}

}  // extern "C"
