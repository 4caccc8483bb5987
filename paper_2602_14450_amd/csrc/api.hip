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

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t spinor_bytes(const Geom& g, int prec) { return spinor_elems(g) * prec_complex_bytes(prec); }
size_t canon_bytes(const Geom& g) { return (size_t)2 * g.Vh * 12 * 16; }
int max_rows(const Geom& g, const DslashTune* tune, int n) {
  int rows = site_grid(g);
  for (int p = 0; p < 3; p++) rows = std::max(rows, flat_rows(g, p));
  for (int p = 0; p < 3; p++) rows = std::max(rows, dslash_partial_rows(g, tune[p], n));
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
  double* partials = nullptr;
  Scalars* sc = nullptr;
  double* history = nullptr;
  int hist_stride = 1;
  double* sums = nullptr;
  double* scale = nullptr;
  size_t bytes = 0;
};

// what: 0 refinement, 1 BiCGStab, 2 operator with canonical layout, 3 preconditioned refinement
Work carve(const qcd_gauge* G, int what, int prec, int max_iter, int n, char* base) {
  const Geom& g = G->g;
  Carve c{base};
  Work w;
  w.n = n;
  if (what == 0 || what == 1 || what == 3) {
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

bool valid_prec(int p) { return p == kFP64 || p == kFP32 || p == kFP16; }

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

// One BiCGStab iteration of Alg. 4 / Alg. 5 for all right-hand sides, entirely on the device.
// With a preconditioner the operator is D c M: v = D (c M p), t = D (c M s), and (t, s) is
// taken against s itself (the TSAux epilogue), so x accumulates the iterate u of D c M u = y.
void bicg_iteration(const qcd_gauge* g, int prec, double kappa, const Work& w, int ftz, const Precond& pc,
                    hipStream_t st) {
  const Geom& G = g->g;
  const int n = w.n;
  const DslashTune& tu = g->tune[prec];
  const int drows = dslash_partial_rows(G, tu, n), frows = flat_rows(G, prec);
  const void* U = g->U[prec];
  launch_p_update(G, prec, n, w.sc, w.p, w.v, w.r, ftz, st);
  if (pc.net) {
    ptc_apply_half(pc.net, n, w.p, w.z, pc.scale, ftz, w.sc, st);
    launch_dslash(prec, G, tu, kOpD, kEpiDotAux, n, w.v, w.z, U, kappa, w.rstar, w.partials, w.sc, ftz, st);
  } else {
    launch_dslash(prec, G, tu, kOpD, kEpiDotAux, n, w.v, w.p, U, kappa, w.rstar, w.partials, w.sc, ftz, st);
  }
  launch_alpha(n, w.sc, w.partials, drows, st);
  launch_s_update(G, prec, n, w.sc, w.r, w.v, ftz, st);
  if (pc.net) {
    ptc_apply_half(pc.net, n, w.r, w.z, pc.scale, ftz, w.sc, st);
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
void residual64(const qcd_gauge* g, double kappa, const Work& w, const Scalars* outer_mask, hipStream_t st) {
  launch_dslash(kFP64, g->g, g->tune[kFP64], kOpD, kEpiResid, w.n, w.r64, w.x64, g->U[kFP64], kappa, w.b64,
                w.partials, outer_mask, 0, st);
}

// Capture one iteration (8 kernels) into a hip graph.  Capture runs on the
// handle's own stream (the null stream cannot be captured); the graph is
// launched on the caller's stream.  The kernels take every changing value
// from device memory, so one capture serves every iteration.
qcd_status iteration_graph(const qcd_gauge* gc, int prec, double kappa, const Work& w, int ftz, const Precond& pc,
                           hipGraphExec_t* out) {
  qcd_gauge* g = const_cast<qcd_gauge*>(gc);
  unsigned long long kbits;
  memcpy(&kbits, &kappa, sizeof kbits);
  unsigned sbits;
  memcpy(&sbits, &pc.scale, sizeof sbits);
  const unsigned long long key[8] = {(unsigned long long)prec, (unsigned long long)w.n, (unsigned long long)w.x,
                                     kbits, (unsigned long long)ftz,
                                     (unsigned long long)(g->tune[prec].sched * 64 + g->tune[prec].variant * 8 +
                                                          g->tune[prec].rhs_tile),
                                     (unsigned long long)(uintptr_t)pc.net, pc.net ? sbits : 0ull};
  if (g->graph_exec && memcmp(key, g->graph_key, sizeof key) == 0) {
    *out = g->graph_exec;
    return QCD_OK;
  }
  if (g->graph_exec) {
    HIP_TRY(hipGraphExecDestroy(g->graph_exec));
    g->graph_exec = nullptr;
  }
  if (!g->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
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

// Run the inner loop from initialised scalars until the device reports a
// stop for every right-hand side; fills the host mirror.  Iterations are
// queued in chunks without host synchronisation (kernels of a stopped solve
// return at once).  After the first chunk, the chunk length is the number of
// iterations the observed convergence rate predicts the slowest right-hand
// side still needs, plus one.
qcd_status bicg_loop(const qcd_gauge* g, int prec, double kappa, const Work& w, const qcd_bicgstab_params& p,
                     const Precond& pc, hipStream_t st) {
  const int K0 = p.check_every > 0 ? p.check_every : 4;
  const int n = w.n;
  qcd_status s = read_scalars(g, w, st);
  if (s) return s;
  hipGraphExec_t gexec = nullptr;
  if (p.use_graph && any_active(g, n)) {
    if ((s = iteration_graph(g, prec, kappa, w, p.ftz, pc, &gexec))) return s;
  }
  int launched = 0, chunk = K0;
  double prev_res2[kMaxRhs];
  int prev_iter[kMaxRhs];
  for (int i = 0; i < n; i++) {
    prev_res2[i] = g->host_sc[i].bnorm2;
    prev_iter[i] = 0;
  }
  while (any_active(g, n) && launched <= p.max_iter + K0) {
    for (int j = 0; j < chunk; j++) {
      if (gexec)
        HIP_TRY(hipGraphLaunch(gexec, st));
      else
        bicg_iteration(g, prec, kappa, w, p.ftz, pc, st);
    }
    HIP_LAUNCHED();
    launched += chunk;
    s = read_scalars(g, w, st);
    if (s) return s;
    chunk = K0;
    if (p.check_every > 0) continue;
    int need_max = 0;
    for (int i = 0; i < n; i++) {
      const Scalars& h = g->host_sc[i];
      if (!h.active || h.iter <= prev_iter[i]) continue;
      const double res2 = h.rnorm2 / (h.gamma_cum * h.gamma_cum);
      const double target = h.tol2 * h.bnorm2;
      const double rate = std::pow(res2 / prev_res2[i], 1.0 / (h.iter - prev_iter[i]));  // per iteration
      int need = K0;
      if (rate > 0.0 && rate < 0.999 && res2 > target)
        need = (int)std::min(64.0, std::max(1.0, std::ceil(std::log(target / res2) / std::log(rate)) + 1.0));
      need_max = std::max(need_max, need);
      prev_res2[i] = res2;
      prev_iter[i] = h.iter;
    }
    if (need_max > 0) chunk = need_max;
  }
  return QCD_OK;
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
  const int flags = prec_mask & ~7;
  prec_mask &= 7;
  if (prec_mask == 0) prec_mask = 7;
  prec_mask |= 1 << kFP64;
  qcd_gauge* g = new qcd_gauge();
  memset(g, 0, sizeof(*g));
  g->g = make_geom(dims);
  // defaults measured on MI355X at 32^3 x 64 (the tuner may override them)
  g->tune[kFP64] = DslashTune{1, 0, 0, 0};
  g->tune[kFP32] = DslashTune{1, 1, 0, 0};
  g->tune[kFP16] = DslashTune{1, 1, 0, 0};
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
    const double thr[3] = {1e-14, 1e-7, 1e-4};
    for (int p = 0; p < 3; p++) g->tune[p].recon = g->su3_dev <= thr[p];
  }
  for (int p = 0; p < 3 && rc == QCD_OK; p++) {
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
  if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  delete g;
  return QCD_OK;
}

qcd_status qcd_set_dslash_tuning(qcd_gauge* g, qcd_prec prec, int sched, int variant, int rhs_tile) {
  if (!g || !valid_prec(prec)) return fail(QCD_ERR_ARG, "invalid handle or precision");
  if (sched < 0 || sched >= kDslashScheds || variant < 0 || variant >= kDslashVariants)
    return fail(QCD_ERR_ARG, "sched must be 0..%d and variant 0..%d", kDslashScheds - 1, kDslashVariants - 1);
  if (rhs_tile != 0 && rhs_tile != 1 && rhs_tile != 2 && rhs_tile != 4)
    return fail(QCD_ERR_ARG, "rhs_tile must be 0 (automatic), 1, 2 or 4");
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
  const int tiles[3] = {1, 2, 4};
  for (int ti = 0; ti < 3; ti++) {
    const int T = tiles[ti];
    if (nrhs % T || (T > 1 && nrhs == 1)) continue;
    for (int sched = 0; sched < kDslashScheds; sched++)
      for (int var = 0; var < (T == 1 ? kDslashVariants : 1); var++) {
        if (sched > 1 && make_sched(g->g, sched, T, nrhs).mode != sched) continue;  // not applicable
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
  if (!g || !valid_prec(prec) || what < 0 || what > 3 || nrhs < 1 || nrhs > kMaxRhs) return 0;
  return carve(g, what, prec, max_iter, nrhs, nullptr).bytes;
}

qcd_status qcd_convert(const qcd_gauge* g, qcd_prec prec, int nrhs, void* native_dev, const void* canonical_dev,
                       double scale, int ftz, double* norm2, void* stream) {
  qcd_status rc = check_gauge(g, kFP64);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!valid_prec(prec) || !native_dev || !canonical_dev) return fail(QCD_ERR_ARG, "invalid argument");
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
  launch_unpack_spinor(g->g, prec, nrhs, (double*)canonical_dev, native_dev, nullptr, scale, S(stream));
  HIP_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_dslash(const qcd_gauge* g, double kappa, qcd_op op, qcd_prec prec, qcd_layout layout, int nrhs,
                      void* out_dev, const void* in_dev, void* stream) {
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!out_dev || !in_dev || out_dev == in_dev) return fail(QCD_ERR_ARG, "out and in must be distinct non-null buffers");
  if (op < QCD_OP_D || op > QCD_OP_HDAG) return fail(QCD_ERR_ARG, "invalid op %d", (int)op);
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  hipStream_t st = S(stream);
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

qcd_status qcd_bicgstab(const qcd_gauge* g, double kappa, qcd_prec prec, int nrhs, void* x_dev, const void* b_dev,
                        const qcd_bicgstab_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const double t0 = now_s();
  qcd_status rc = check_gauge(g, prec);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!x_dev || !b_dev) return fail(QCD_ERR_ARG, "null vector");
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if ((rc = check_bicg_params(p))) return rc;
  hipStream_t st = S(stream);
  Work w;
  if ((rc = get_work(g, 1, prec, p->max_iter, nrhs, ws, ws_bytes, &w))) return rc;
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

qcd_status qcd_solve_mixed_ir(const qcd_gauge* g, double kappa, int nrhs, void* x_dev, const void* b_dev,
                              const qcd_ir_params* p, qcd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const double t0 = now_s();
  if (!p) return fail(QCD_ERR_ARG, "null parameters");
  qcd_status rc = check_gauge(g, p->inner_prec);
  if (rc) return rc;
  if ((rc = check_nrhs(nrhs))) return rc;
  if (!x_dev || !b_dev) return fail(QCD_ERR_ARG, "null vector");
  if (!(kappa > 0)) return fail(QCD_ERR_ARG, "kappa must be > 0");
  if (!(p->tol > 0) || p->max_outer <= 0 || !(p->s > 0)) return fail(QCD_ERR_ARG, "tol > 0, max_outer > 0, s > 0 required");
  if ((rc = check_bicg_params(&p->inner))) return rc;
  const int prec = p->inner_prec;
  const int n = nrhs;
  qcd_ptc* net = const_cast<qcd_ptc*>(p->precond);
  if (net) {
    if (prec != kFP16) return fail(QCD_ERR_UNSUPPORTED, "the network preconditioner runs with the FP16 inner solve");
    if (ptc_gauge(net) != g) return fail(QCD_ERR_ARG, "the network is bound to another gauge handle");
    if (n > ptc_max_batch(net)) return fail(QCD_ERR_ARG, "nrhs %d exceeds the network's max_batch %d", n,
                                            ptc_max_batch(net));
    if (!(p->precond_scale >= 0) || !std::isfinite(p->precond_scale))
      return fail(QCD_ERR_ARG, "precond_scale must be finite and >= 0");
  }
  hipStream_t st = S(stream);
  Work w;
  if ((rc = get_work(g, net ? 3 : 0, prec, p->inner.max_iter, n, ws, ws_bytes, &w))) return rc;
  const Geom& G = g->g;
  const int rows = site_grid(G);
  const int drows64 = dslash_partial_rows(G, g->tune[kFP64], n);
  Scalars hs[kMaxRhs];
  for (int i = 0; i < n; i++) {
    init_params(&hs[i], p->inner);
    hs[i].out_tol = p->tol;
  }
  HIP_TRY(hipMemcpyAsync(w.sc, hs, sizeof(Scalars) * n, hipMemcpyHostToDevice, st));
  // b in the native FP64 layout; r = b, x = 0
  launch_pack_spinor(G, kFP64, n, w.b64, (const double*)b_dev, 1.0, 0, w.partials, st);
  launch_outer_residual_norm(n, w.sc, w.partials, rows, p->s, st);
  HIP_TRY(hipMemcpyAsync(w.r64, w.b64, n * spinor_bytes(G, kFP64), hipMemcpyDeviceToDevice, st));
  launch_zero(G, kFP64, n, w.x64, st);
  HIP_LAUNCHED();
  if ((rc = read_scalars(g, w, st))) return rc;
  double bn[kMaxRhs], rn[kMaxRhs];
  int outer[kMaxRhs], inner_total[kMaxRhs], last_status[kMaxRhs];
  qcd_status result[kMaxRhs];
  bool any = false;
  for (int i = 0; i < n; i++) {
    bn[i] = rn[i] = g->host_sc[i].out_rnorm;
    outer[i] = inner_total[i] = 0;
    last_status[i] = kConverged;
    result[i] = QCD_OK;
    if (!std::isfinite(bn[i])) result[i] = fail(QCD_ERR_ARG, "non-finite right-hand side %d", i);
    if (info) {
      info[i].history_len = 0;
      info[i].first_shat_over_s = 0;
      info[i].precond_steps = 0;
      info[i].precond_fallback = -1;
      info[i].precond_scale = 0;
    }
    any |= g->host_sc[i].outer_active && std::isfinite(bn[i]);
  }
  if (!std::isfinite(bn[0]) && n == 1) any = false;
  Precond pc;
  pc.net = net;
  pc.scale = (float)p->precond_scale;
  int pc_steps = 0, pc_fallback = -1;
  int step = 0;
  while (any) {
    if (step >= p->max_outer) {
      for (int i = 0; i < n; i++)
        if (g->host_sc[i].outer_active) result[i] = worse(result[i], QCD_NOT_CONVERGED);
      break;
    }
    // keep x so that a preconditioned step that fails can be undone
    if (pc.net) HIP_TRY(hipMemcpyAsync(w.x64b, w.x64, n * spinor_bytes(G, kFP64), hipMemcpyDeviceToDevice, st));
    // y~ = low(r s/|r|), s^ = |single(y~)|, inner solver start (right-hand
    // sides that met the tolerance are skipped by the kernels)
    launch_convert(G, prec, n, w.sc, (const double*)w.r64, w.r, w.rstar, w.partials, p->inner.ftz, st);
    launch_convert_finish(n, w.sc, w.partials, rows, p->recalc_shat, p->s, st);
    HIP_LAUNCHED();
    if (pc.net && pc.scale == 0.0f) {  // c = 1 / gain of M, measured on the first y~
      double gain = 0;
      if ((rc = ptc_gain(pc.net, n, w.r, &gain, st))) return rc;
      pc.scale = gain > 0 ? (float)(1.0 / gain) : 1.0f;
    }
    if ((rc = bicg_loop(g, prec, kappa, w, p->inner, pc, st))) return rc;
    Scalars sc[kMaxRhs];
    memcpy(sc, g->host_sc, sizeof(Scalars) * n);
    bool inner_failed[kMaxRhs];
    for (int i = 0; i < n; i++) {
      inner_failed[i] = false;
      if (!sc[i].outer_active) continue;
      if (info && outer[i] == 0) info[i].first_shat_over_s = sc[i].shat / p->s;
      if (info && info[i].zeros && outer[i] < info[i].outer_history_cap) info[i].zeros[outer[i]] = sc[i].zeros;
      copy_history(info ? info + i : nullptr, w, i, sc[i].iter, sc[i].bnorm2, st);
      inner_total[i] += sc[i].iter;
      last_status[i] = sc[i].status;
      inner_failed[i] = sc[i].status == kNonFinite || sc[i].iter == 0;
      if (inner_failed[i] && !pc.net)
        result[i] = fail(sc[i].status == kNonFinite ? QCD_ERR_NONFINITE : QCD_ERR_BREAKDOWN,
                         "inner solve of right-hand side %d failed (status %d) in refinement step %d", i,
                         sc[i].status, outer[i]);
    }
    // x += (|r| / s^) double(t~), with t~ = c M u~ when preconditioned; r = b - D x
    // in FP64 (skipped where not refining)
    if (pc.net) {
      ptc_apply_half(pc.net, n, w.x, w.z, pc.scale, p->inner.ftz, nullptr, st);
      launch_correct(G, prec, n, w.sc, (double*)w.x64, w.z, st);
    } else {
      launch_correct(G, prec, n, w.sc, (double*)w.x64, w.x, st);
    }
    residual64(g, kappa, w, nullptr, st);
    launch_outer_residual_norm(n, w.sc, w.partials, drows64, p->s, st);
    HIP_LAUNCHED();
    if ((rc = read_scalars(g, w, st))) return rc;
    if (pc.net) {
      // flexible step accepted only if every refining residual dropped and stayed finite
      bool undo = false;
      for (int i = 0; i < n; i++) {
        if (!sc[i].outer_active) continue;
        const double r_new = g->host_sc[i].out_rnorm;
        if (inner_failed[i] || !std::isfinite(r_new) || !(r_new < rn[i])) undo = true;
      }
      if (undo) {
        // restore x of the right-hand sides whose step failed, recompute r, and go on without M
        for (int i = 0; i < n; i++) {
          if (!sc[i].outer_active) continue;
          const double r_new = g->host_sc[i].out_rnorm;
          if (inner_failed[i] || !std::isfinite(r_new) || !(r_new < rn[i]))
            HIP_TRY(hipMemcpyAsync((char*)w.x64 + i * spinor_bytes(G, kFP64), (char*)w.x64b + i * spinor_bytes(G, kFP64),
                                   spinor_bytes(G, kFP64), hipMemcpyDeviceToDevice, st));
        }
        for (int i = 0; i < n; i++) g->host_sc[i].outer_active = sc[i].outer_active;
        HIP_TRY(hipMemcpyAsync(w.sc, g->host_sc, sizeof(Scalars) * n, hipMemcpyHostToDevice, st));
        residual64(g, kappa, w, nullptr, st);
        launch_outer_residual_norm(n, w.sc, w.partials, drows64, p->s, st);
        HIP_LAUNCHED();
        if ((rc = read_scalars(g, w, st))) return rc;
        pc_fallback = step;
        pc.net = nullptr;
      } else {
        pc_steps++;
      }
    }
    any = false;
    for (int i = 0; i < n; i++) {
      if (!sc[i].outer_active) continue;
      outer[i]++;
      rn[i] = g->host_sc[i].out_rnorm;
      if (info && info[i].outer_history && outer[i] - 1 < info[i].outer_history_cap)
        info[i].outer_history[outer[i] - 1] = rn[i] / bn[i];
      if (!std::isfinite(rn[i])) result[i] = fail(QCD_ERR_NONFINITE, "non-finite outer residual");
      if (result[i] < 0) {  // stop refining this right-hand side
        g->host_sc[i].outer_active = 0;
        HIP_TRY(hipMemcpyAsync(&w.sc[i].outer_active, &g->host_sc[i].outer_active, sizeof(int),
                               hipMemcpyHostToDevice, st));
      }
      any |= g->host_sc[i].outer_active != 0;
    }
    step++;
  }
  launch_unpack_spinor(G, kFP64, n, (double*)x_dev, w.x64, nullptr, 1.0, st);
  HIP_LAUNCHED();
  HIP_TRY(hipStreamSynchronize(st));
  qcd_status res = QCD_OK;
  for (int i = 0; i < n; i++) {
    if (info) {
      info[i].outer_iters = outer[i];
      info[i].inner_iters = inner_total[i];
      info[i].matvec_low = 2 * inner_total[i];
      info[i].matvec_fp64 = outer[i];
      info[i].true_rel_residual = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
      info[i].inner_status = last_status[i];
      info[i].seconds = now_s() - t0;
      info[i].precond_steps = pc_steps;
      info[i].precond_fallback = pc_fallback;
      info[i].precond_scale = net ? pc.scale : 0.0;
    }
    res = worse(res, result[i]);
  }
  return res;
}

}  // extern "C"
