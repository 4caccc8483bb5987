// Streaming vector kernels of the rescaled BiCGStab (Alg. 4 / Alg. 5) and
// the rescaled iterative refinement (Alg. 2 / Alg. 3), plus layout and
// precision conversions.  One thread handles the 12 complex components of
// one site; every wave-wide access is a contiguous run of the native layout.
// Reductions are formed from the stored values and written as per-block FP64
// partials; the single-block finish kernels sum them in a fixed order and
// advance the FP64 scalar recurrences held in device memory.
#include "common.h"
#include "internal.h"

namespace qcd {

static inline int nbp_of(const Geom& g) { return (g.Vh + 255) / 256; }
int site_grid(const Geom& g) { return 2 * nbp_of(g); }

struct SiteId { int par, h; bool valid; };
__device__ __forceinline__ SiteId site_id(const Geom& g) {
  const int nbp = (g.Vh + 255) / 256;
  SiteId s;
  s.par = blockIdx.x / nbp;
  s.h = (blockIdx.x % nbp) * 256 + threadIdx.x;
  s.valid = s.h < g.Vh;
  return s;
}
__device__ __forceinline__ int64_t lex_site(const Geom& g, int par, int h) {
  Coord c = decode(g, par, h);
  return c.x + (int64_t)g.L[0] * (c.y + (int64_t)g.L[1] * (c.z + (int64_t)g.L[2] * c.t));
}

// ---------------------------------------------------------------------------
// Layout conversions

template <typename S>
__global__ __launch_bounds__(256) void k_pack_links(Geom g, S* __restrict__ dst, const double* __restrict__ Uc) {
  SiteId id = site_id(g);
  if (!id.valid) return;
  const int64_t s = lex_site(g, id.par, id.h);
  for (int mu = 0; mu < 4; mu++)
    for (int k = 0; k < 9; k++) {
      const double* src = Uc + ((s * 4 + mu) * 9 + k) * 2;
      dst[lk_index(g, mu, id.par, id.h, k)] = pack_from_double<S>(src[0], src[1], 0);
    }
}

// dst = round(scale * canon); partial |dst|^2 per block (from stored values).
template <typename S>
__global__ __launch_bounds__(256) void k_pack_spinor(Geom g, S* __restrict__ dst, const double* __restrict__ src,
                                                     double scale, int ftz, double* __restrict__ partials) {
  using T = typename Traits<S>::T;
  SiteId id = site_id(g);
  double red[1] = {0.0};
  if (id.valid) {
    const int64_t s = lex_site(g, id.par, id.h);
    T acc = 0;
    for (int k = 0; k < 12; k++) {
      const S v = pack_from_double<S>(scale * src[(s * 12 + k) * 2], scale * src[(s * 12 + k) * 2 + 1], ftz);
      dst[sp_index(g, id.par, id.h, k)] = v;
      acc += norm2(Traits<S>::load(&v));
    }
    red[0] = acc;
  }
  if (partials) block_reduce_store<1>(red, partials, blockIdx.x);
}

template <typename S>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geom g, double* __restrict__ dst, const S* __restrict__ src,
                                                       double scale) {
  SiteId id = site_id(g);
  if (!id.valid) return;
  const int64_t s = lex_site(g, id.par, id.h);
  for (int k = 0; k < 12; k++) {
    const auto v = Traits<S>::load(src + sp_index(g, id.par, id.h, k));
    dst[(s * 12 + k) * 2] = scale * (double)v.re;
    dst[(s * 12 + k) * 2 + 1] = scale * (double)v.im;
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_zero(Geom g, S* __restrict__ dst) {
  SiteId id = site_id(g);
  if (!id.valid) return;
  using T = typename Traits<S>::T;
  for (int k = 0; k < 12; k++) dst[sp_index(g, id.par, id.h, k)] = Traits<S>::pack(cx<T>(0, 0), 0);
}

// ---------------------------------------------------------------------------
// BiCGStab body (Alg. 4 / Alg. 5).  Vectors: x, r (holds s between the two
// matrix applications), r*, p, v, t.

// p := beta (p - omega' v) + r, with the previous iteration's rescaling of
// p and v by gamma folded into the coefficient (pcoef = beta * gamma).  In
// the first iteration p = r (p = v = 0 initially).
template <typename S>
__global__ __launch_bounds__(256) void k_p_update(Geom g, const Scalars* __restrict__ sc, S* __restrict__ p,
                                                  const S* __restrict__ v, const S* __restrict__ r, int ftz) {
  using T = typename Traits<S>::T;
  if (!sc->active) return;
  SiteId id = site_id(g);
  if (!id.valid) return;
  const int first = sc->first;
  const cx<T> c((T)sc->pcoef[0], (T)sc->pcoef[1]);
  const cx<T> w((T)sc->omega_prev[0], (T)sc->omega_prev[1]);
  for (int k = 0; k < 12; k++) {
    const size_t i = sp_index(g, id.par, id.h, k);
    cx<T> rv = Traits<S>::load(r + i);
    cx<T> o = rv;
    if (!first) o = c * (Traits<S>::load(p + i) - w * Traits<S>::load(v + i)) + rv;
    p[i] = Traits<S>::pack(o, ftz);
  }
}

// r := r - alpha v   (the vector s of the standard formulation)
template <typename S>
__global__ __launch_bounds__(256) void k_s_update(Geom g, const Scalars* __restrict__ sc, S* __restrict__ r,
                                                  const S* __restrict__ v, int ftz) {
  using T = typename Traits<S>::T;
  if (!sc->active) return;
  SiteId id = site_id(g);
  if (!id.valid) return;
  const cx<T> a((T)sc->alpha[0], (T)sc->alpha[1]);
  for (int k = 0; k < 12; k++) {
    const size_t i = sp_index(g, id.par, id.h, k);
    r[i] = Traits<S>::pack(Traits<S>::load(r + i) - a * Traits<S>::load(v + i), ftz);
  }
}

// x := xscale x + (lambda'/gamma') (omega s + alpha p);
// r := gamma_pred (s - omega t), stored in the buffer that held s.
// Partials (from the values as stored): |s - omega t|^2 before the rescaling
// (FP32/FP64 arithmetic, unrounded), |r|^2, (r*, r) and |x|^2.
template <typename S>
__global__ __launch_bounds__(256) void k_xr_update(Geom g, const Scalars* __restrict__ sc, S* __restrict__ x,
                                                   S* __restrict__ r, const S* __restrict__ t,
                                                   const S* __restrict__ p, const S* __restrict__ rstar,
                                                   double* __restrict__ partials, int ftz) {
  using T = typename Traits<S>::T;
  if (!sc->active) return;
  SiteId id = site_id(g);
  double red[5] = {0, 0, 0, 0, 0};
  if (id.valid) {
    const int first = sc->first;
    const T xs = (T)sc->xscale, xc = (T)sc->xcoef, gp = (T)sc->gamma_pred;
    const cx<T> om((T)sc->omega[0], (T)sc->omega[1]);
    const cx<T> al((T)sc->alpha[0], (T)sc->alpha[1]);
    T ww = 0, rr = 0, rsr_re = 0, rsr_im = 0, xx = 0;
    for (int k = 0; k < 12; k++) {
      const size_t i = sp_index(g, id.par, id.h, k);
      const cx<T> s = Traits<S>::load(r + i);
      const cx<T> pk = Traits<S>::load(p + i);
      cx<T> xn = xc * (om * s + al * pk);
      if (!first) xn = xs * Traits<S>::load(x + i) + xn;
      const S xst = Traits<S>::pack(xn, ftz);
      x[i] = xst;
      const cx<T> w = s - om * Traits<S>::load(t + i);
      const S rst = Traits<S>::pack(gp * w, ftz);
      r[i] = rst;
      const cx<T> rs = Traits<S>::load(&rst), xsv = Traits<S>::load(&xst);
      const cx<T> q = Traits<S>::load(rstar + i);
      ww += norm2(w);
      rr += norm2(rs);
      rsr_re += q.re * rs.re + q.im * rs.im;
      rsr_im += q.re * rs.im - q.im * rs.re;
      xx += norm2(xsv);
    }
    red[0] = ww; red[1] = rr; red[2] = rsr_re; red[3] = rsr_im; red[4] = xx;
  }
  block_reduce_store<5>(red, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Refinement step (Alg. 3): y~ = low(scale * r) with scale = s / |r|;
// the inner solver starts from r = r* = y~.  Partials: sum single(y~)^2 in
// the arithmetic precision per site (FP64 across sites), and the number of
// zero reals in y~ (the underflow diagnostic of Fig. 9).
template <typename S>
__global__ __launch_bounds__(256) void k_convert(Geom g, const Scalars* __restrict__ sc, const double2* __restrict__ r64,
                                                 S* __restrict__ y, S* __restrict__ rstar,
                                                 double* __restrict__ partials, int ftz) {
  using T = typename Traits<S>::T;
  SiteId id = site_id(g);
  double red[2] = {0, 0};
  if (id.valid) {
    const double sc_ = sc->out_scale;
    T acc = 0;
    int zeros = 0;
    for (int k = 0; k < 12; k++) {
      const size_t i = sp_index(g, id.par, id.h, k);
      const double2 v = r64[i];
      const S st = pack_from_double<S>(sc_ * v.x, sc_ * v.y, ftz);
      y[i] = st;
      rstar[i] = st;
      const cx<T> f = Traits<S>::load(&st);
      acc += norm2(f);
      zeros += (f.re == (T)0) + (f.im == (T)0);
    }
    red[0] = acc;
    red[1] = zeros;
  }
  block_reduce_store<2>(red, partials, blockIdx.x);
}

// x64 := x64 + (|r| / s^) * double(x_inner), with x_inner = xscale * X / lambda'.
template <typename S>
__global__ __launch_bounds__(256) void k_correct(Geom g, const Scalars* __restrict__ sc, double2* __restrict__ x64,
                                                 const S* __restrict__ xlo) {
  SiteId id = site_id(g);
  if (!id.valid) return;
  const double c = sc->out_rnorm / sc->shat * sc->xscale / sc->lambda_cum;
  for (int k = 0; k < 12; k++) {
    const size_t i = sp_index(g, id.par, id.h, k);
    const auto v = Traits<S>::load(xlo + i);
    double2 o = x64[i];
    o.x += c * (double)v.re;
    o.y += c * (double)v.im;
    x64[i] = o;
  }
}

// ---------------------------------------------------------------------------
// Finish kernels: one block sums the partial rows, thread 0 updates scalars.

__device__ __forceinline__ cx<double> cd(const double* a) { return cx<double>(a[0], a[1]); }
__device__ __forceinline__ void setc(double* a, cx<double> v) { a[0] = v.re; a[1] = v.im; }
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return cx<double>((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__device__ __forceinline__ bool finite_c(cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

__device__ void stop(Scalars* sc, int status) {
  sc->status = status;
  sc->active = 0;
}

// Start of a BiCGStab run: x0 = 0, r = r* = b, p = v = 0, rho' = |r|^2,
// omega' = alpha' = gamma' = lambda' = 1.
__device__ void bicg_init_dev(Scalars* sc, double bn2) {
  sc->bnorm2 = bn2;
  sc->rnorm2 = bn2;
  sc->rho[0] = bn2; sc->rho[1] = 0;
  sc->rho_prev[0] = bn2; sc->rho_prev[1] = 0;
  sc->alpha_prev[0] = 1; sc->alpha_prev[1] = 0;
  sc->omega_prev[0] = 1; sc->omega_prev[1] = 0;
  sc->beta[0] = 1; sc->beta[1] = 0;
  sc->pcoef[0] = 0; sc->pcoef[1] = 0;
  sc->gamma = sc->gamma_cum = sc->lambda_cum = 1.0;
  sc->xscale = 1.0;
  sc->xcoef = 1.0;
  sc->gamma_pred = 1.0;
  sc->iter = 0;
  sc->first = 1;
  sc->status = kRunning;
  sc->active = 1;
  if (!(bn2 > 0.0)) stop(sc, bn2 == 0.0 ? kConverged : kNonFinite);
  else if (bn2 <= sc->tol2 * bn2) stop(sc, kConverged);
}

__global__ void k_bicg_init(Scalars* sc, const double* partials, int nrows) {
  double s[1];
  finish_sum<1>(partials, nrows, s);
  if (threadIdx.x == 0) bicg_init_dev(sc, s[0]);
}

// alpha = rho / (r*, v)
__global__ void k_alpha(Scalars* sc, const double* partials, int nrows) {
  if (!sc->active) return;
  double s[2];
  finish_sum<2>(partials, nrows, s);
  if (threadIdx.x != 0) return;
  const cx<double> rv(s[0], s[1]);
  if (rv.re == 0.0 && rv.im == 0.0) { stop(sc, kBreakdown); return; }
  const cx<double> a = cdiv(cd(sc->rho), rv);
  if (!finite_c(a)) { stop(sc, kNonFinite); return; }
  setc(sc->alpha, a);
}

// omega = (t,s)/(t,t) with the omega_0 prescription; the x-update factor
// lambda'/gamma'; and the factor that rescales the new residual to norm
// sigma, from |s - omega t|^2 = (s,s) - 2 Re(conj(omega)(t,s)) + |omega|^2 (t,t).
__global__ void k_omega(Scalars* sc, const double* partials, int nrows) {
  if (!sc->active) return;
  double s[4];
  finish_sum<4>(partials, nrows, s);
  if (threadIdx.x != 0) return;
  const cx<double> ts(s[0], s[1]);
  const double tt = s[2], ss = s[3];
  if (!(tt > 0.0)) {  // t = A s = 0 means s = 0: the previous step solved the system
    if (ss == 0.0) {
      sc->omega[0] = 0; sc->omega[1] = 0;
    } else { stop(sc, kBreakdown); return; }
  } else {
    cx<double> om = (1.0 / tt) * ts;
    const double ah = sqrt(ts.re * ts.re + ts.im * ts.im) / sqrt(tt * ss);
    if (ah < sc->omega0) om = (sc->omega0 / ah) * om;
    setc(sc->omega, om);
  }
  const cx<double> om = cd(sc->omega);
  sc->xcoef = sc->lambda_cum / sc->gamma_cum;
  if (sc->sigma > 0.0) {
    double g2 = ss - 2.0 * (om.re * ts.re + om.im * ts.im) + (om.re * om.re + om.im * om.im) * tt;
    // below ~1e-6 (s,s) the prediction is dominated by cancellation; the
    // floor keeps the stored residual from overflowing in that case, and
    // the recalculated gamma (or the factor itself) keeps the bookkeeping exact
    const double floor2 = 1e-10 * ss;
    if (!(g2 > floor2)) g2 = floor2;
    sc->gamma_pred = (g2 > 0.0) ? sc->sigma / sqrt(g2) : 1.0;
  } else {
    sc->gamma_pred = 1.0;
  }
  if (!finite_c(om) || !isfinite(sc->gamma_pred)) stop(sc, kNonFinite);
}

// End of an iteration: gamma (applied or recalculated), rho' = gamma rho,
// gamma' *= gamma, the next rho and beta, lambda for Alg. 5, the stopping test.
__global__ void k_iter_end(Scalars* sc, const double* partials, int nrows, double* history) {
  if (!sc->active) return;
  double s[5];
  finish_sum<5>(partials, nrows, s);
  if (threadIdx.x != 0) return;
  const double ww = s[0], rr = s[1], xx = s[4];
  const cx<double> rsr(s[2], s[3]);
  double gamma = 1.0;
  if (sc->sigma > 0.0) {
    if (sc->recalc_gamma) gamma = (ww > 0.0) ? sqrt(rr / ww) : sc->gamma_pred;
    else gamma = sc->gamma_pred;
  }
  sc->gamma = gamma;
  const cx<double> rho_cur = cd(sc->rho);
  setc(sc->rho_prev, gamma * rho_cur);
  setc(sc->omega_prev, cd(sc->omega));
  setc(sc->alpha_prev, cd(sc->alpha));
  sc->gamma_cum *= gamma;
  setc(sc->rho, rsr);
  // beta for the next iteration and the folded p/v rescaling
  const cx<double> beta = cdiv(rsr * cd(sc->alpha_prev), cd(sc->rho_prev) * cd(sc->omega_prev));
  setc(sc->beta, beta);
  setc(sc->pcoef, gamma * beta);
  // Alg. 5: lambda = sigma_lambda / |x|, applied to x at the next update
  if (sc->sigma_lambda > 0.0 && xx > 0.0) {
    const double lam = sc->sigma_lambda / sqrt(xx);
    sc->xscale = lam;
    sc->lambda_cum *= lam;
  } else {
    sc->xscale = 1.0;
  }
  sc->rnorm2 = rr;
  sc->first = 0;
  const double res2 = rr / (sc->gamma_cum * sc->gamma_cum);
  if (history && sc->iter < sc->max_iter) history[sc->iter] = res2;
  sc->iter += 1;
  if (!isfinite(res2) || !finite_c(beta) || !isfinite(sc->lambda_cum) || !isfinite(sc->gamma_cum)) {
    // an exact zero residual ends the run as converged
    if (rr == 0.0 && ww == 0.0) stop(sc, kConverged);
    else stop(sc, kNonFinite);
    return;
  }
  if (res2 <= sc->tol2 * sc->bnorm2) { stop(sc, kConverged); return; }
  if (rsr.re == 0.0 && rsr.im == 0.0) { stop(sc, kBreakdown); return; }
  if (sc->iter >= sc->max_iter) stop(sc, kMaxIter);
}

// Outer step: |r| of the FP64 residual and the rescaling factor s / |r|.
__global__ void k_outer_norm(Scalars* sc, const double* partials, int nrows, double s_target) {
  double s[1];
  finish_sum<1>(partials, nrows, s);
  if (threadIdx.x != 0) return;
  sc->out_rnorm = sqrt(s[0]);
  sc->out_scale = (s[0] > 0.0) ? s_target / sc->out_rnorm : 0.0;
}

// After the conversion: s^ (Alg. 3) and the start of the inner BiCGStab.
__global__ void k_convert_finish(Scalars* sc, const double* partials, int nrows, int recalc_shat, double s_target) {
  double s[2];
  finish_sum<2>(partials, nrows, s);
  if (threadIdx.x != 0) return;
  sc->shat = recalc_shat ? sqrt(s[0]) : s_target;
  sc->zeros = s[1];
  bicg_init_dev(sc, s[0]);
}

__global__ void k_finish_sum_any(const double* partials, int nrows, int nv, double* out) {
  // generic: sums up to 8 columns (used for norms the host asks for)
  double acc[8];
  for (int i = 0; i < 8; i++) acc[i] = 0;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x)
    for (int i = 0; i < nv; i++) acc[i] += partials[(size_t)r * nv + i];
  __shared__ double red[8][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = 0; i < 8; i++) {
    double a = acc[i];
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) red[i][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < nv; i++) {
      double s = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[i][w];
      out[i] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers

#define QCD_DISPATCH(prec, FN, ...)                     \
  do {                                                  \
    if ((prec) == kFP64) FN<double2>(__VA_ARGS__);      \
    else if ((prec) == kFP32) FN<float2>(__VA_ARGS__);  \
    else FN<__half2>(__VA_ARGS__);                      \
  } while (0)

template <typename S> static void pack_links_t(const Geom& g, void* dst, const double* U, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_links<S>, dim3(site_grid(g)), dim3(256), 0, st, g, (S*)dst, U);
}
void launch_pack_links(const Geom& g, int prec, void* dst, const double* U, hipStream_t st) {
  QCD_DISPATCH(prec, pack_links_t, g, dst, U, st);
}

template <typename S>
static void pack_spinor_t(const Geom& g, void* dst, const double* c, double scale, int ftz, double* partials,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_pack_spinor<S>, dim3(site_grid(g)), dim3(256), 0, st, g, (S*)dst, c, scale, ftz, partials);
}
void launch_pack_spinor(const Geom& g, int prec, void* dst, const double* canon, double scale, int ftz,
                        double* partials, hipStream_t st) {
  QCD_DISPATCH(prec, pack_spinor_t, g, dst, canon, scale, ftz, partials, st);
}

template <typename S>
static void unpack_spinor_t(const Geom& g, double* c, const void* src, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_spinor<S>, dim3(site_grid(g)), dim3(256), 0, st, g, c, (const S*)src, scale);
}
void launch_unpack_spinor(const Geom& g, int prec, double* canon, const void* src, double scale, hipStream_t st) {
  QCD_DISPATCH(prec, unpack_spinor_t, g, canon, src, scale, st);
}

template <typename S> static void zero_t(const Geom& g, void* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<S>, dim3(site_grid(g)), dim3(256), 0, st, g, (S*)dst);
}
void launch_zero(const Geom& g, int prec, void* dst, hipStream_t st) { QCD_DISPATCH(prec, zero_t, g, dst, st); }

void launch_bicg_init(Scalars* sc, const double* partials, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_bicg_init, dim3(1), dim3(1024), 0, st, sc, partials, nrows);
}

template <typename S>
static void p_update_t(const Geom& g, Scalars* sc, void* p, const void* v, const void* r, int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_p_update<S>, dim3(site_grid(g)), dim3(256), 0, st, g, sc, (S*)p, (const S*)v, (const S*)r,
                     ftz);
}
void launch_p_update(const Geom& g, int prec, Scalars* sc, void* p, const void* v, const void* r, int ftz,
                     hipStream_t st) {
  QCD_DISPATCH(prec, p_update_t, g, sc, p, v, r, ftz, st);
}

void launch_alpha(Scalars* sc, const double* partials, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(1024), 0, st, sc, partials, nrows);
}

template <typename S>
static void s_update_t(const Geom& g, Scalars* sc, void* r, const void* v, int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_s_update<S>, dim3(site_grid(g)), dim3(256), 0, st, g, sc, (S*)r, (const S*)v, ftz);
}
void launch_s_update(const Geom& g, int prec, Scalars* sc, void* r, const void* v, int ftz, hipStream_t st) {
  QCD_DISPATCH(prec, s_update_t, g, sc, r, v, ftz, st);
}

void launch_omega(Scalars* sc, const double* partials, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_omega, dim3(1), dim3(1024), 0, st, sc, partials, nrows);
}

template <typename S>
static void xr_update_t(const Geom& g, Scalars* sc, void* x, void* r, const void* t, const void* p, const void* rs,
                        double* partials, int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_xr_update<S>, dim3(site_grid(g)), dim3(256), 0, st, g, sc, (S*)x, (S*)r, (const S*)t,
                     (const S*)p, (const S*)rs, partials, ftz);
}
void launch_xr_update(const Geom& g, int prec, Scalars* sc, void* x, void* r, const void* t, const void* p,
                      const void* rstar, double* partials, int ftz, hipStream_t st) {
  QCD_DISPATCH(prec, xr_update_t, g, sc, x, r, t, p, rstar, partials, ftz, st);
}

void launch_iter_end(Scalars* sc, const double* partials, int nrows, double* history, hipStream_t st) {
  hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(1024), 0, st, sc, partials, nrows, history);
}

void launch_outer_residual_norm(Scalars* sc, const double* partials, int nrows, double s_target, hipStream_t st) {
  hipLaunchKernelGGL(k_outer_norm, dim3(1), dim3(1024), 0, st, sc, partials, nrows, s_target);
}

template <typename S>
static void convert_t(const Geom& g, Scalars* sc, const double* r64, void* y, void* rstar, double* partials, int ftz,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_convert<S>, dim3(site_grid(g)), dim3(256), 0, st, g, sc, (const double2*)r64, (S*)y,
                     (S*)rstar, partials, ftz);
}
void launch_convert(const Geom& g, int prec, Scalars* sc, const double* r64, void* y, void* rstar, void*,
                    double* partials, int ftz, hipStream_t st) {
  QCD_DISPATCH(prec, convert_t, g, sc, r64, y, rstar, partials, ftz, st);
}

void launch_convert_finish(Scalars* sc, const double* partials, int nrows, int recalc_shat, double s_target,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_convert_finish, dim3(1), dim3(1024), 0, st, sc, partials, nrows, recalc_shat, s_target);
}

template <typename S>
static void correct_t(const Geom& g, Scalars* sc, double* x64, const void* xlo, hipStream_t st) {
  hipLaunchKernelGGL(k_correct<S>, dim3(site_grid(g)), dim3(256), 0, st, g, sc, (double2*)x64, (const S*)xlo);
}
void launch_correct(const Geom& g, int prec, Scalars* sc, double* x64, const void* xlo, hipStream_t st) {
  QCD_DISPATCH(prec, correct_t, g, sc, x64, xlo, st);
}

void launch_finish_sum(const double* partials, int nrows, int nv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_sum_any, dim3(1), dim3(1024), 0, st, partials, nrows, nv, out);
}

}  // namespace qcd
