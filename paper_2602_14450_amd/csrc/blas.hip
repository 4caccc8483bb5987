// Streaming vector kernels of the rescaled BiCGStab (Alg. 4 / Alg. 5) and
// the rescaled iterative refinement (Alg. 2 / Alg. 3), plus layout and
// precision conversions, for n right-hand sides at once (grid.y indexes the
// right-hand side; vectors are n native spinors back to back).  Reductions
// are formed from the stored values and written as per-block FP64 partials;
// the finish kernels (one block per right-hand side) sum them in a fixed
// order and advance the FP64 scalar recurrences held in device memory.
#include "common.h"
#include "internal.h"

#include <algorithm>

namespace qcd {

// Site-ordered kernels (layout / precision conversions) use one thread per
// site; the BLAS-1 kernels walk each native vector as a flat array of
// 16-byte granules with a fixed grid, so their partial-sum rows number at
// most kFlatBlocks per right-hand side.
constexpr int kFlatBlocks = 1024;
int site_grid(const Geom& g) { return (g.npar * g.Vh + 255) / 256; }
template <typename S> static int flat_grid(const Geom& g) {
  const size_t n = spinor_granules<S>(g);
  const size_t b = (n + 255) / 256;
  return (int)(b < (size_t)kFlatBlocks ? b : (size_t)kFlatBlocks);
}
int flat_rows(const Geom& g, int prec) {
  return prec == kFP64 ? flat_grid<double2>(g) : (prec == kFP32 ? flat_grid<float2>(g) : flat_grid<__half2>(g));  // BF16 as FP16
}

struct SiteId { int par, h; bool valid; };
__device__ __forceinline__ SiteId site_id(const Geom& g) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  SiteId s;
  s.par = g.npar == 2 && i >= g.Vh;
  s.h = i - s.par * g.Vh;
  s.valid = i < g.npar * g.Vh;
  return s;
}
__device__ __forceinline__ int64_t lex_site(const Geom& g, int par, int h) {
  Coord c = decode(g, par, h);
  return c.x + (int64_t)g.L[0] * (c.y + (int64_t)g.L[1] * (c.z + (int64_t)g.L[2] * c.t));
}
__device__ __forceinline__ int64_t volume(const Geom& g) { return 2 * (int64_t)g.Vh; }

// ---------------------------------------------------------------------------
// Layout conversions

template <typename S, int NE>
__global__ __launch_bounds__(256) void k_pack_links(Geom g, S* __restrict__ dst, const double* __restrict__ Uc) {
  SiteId id = site_id(g);
  if (!id.valid) return;
  const int64_t s = lex_site(g, id.par, id.h);
  const int lane = id.h & 63;
  for (int mu = 0; mu < 4; mu++) {
    S* b = dst + lk_block<NE>(g, mu, id.par, id.h);
    for (int k = 0; k < NE; k++) {
      const double* src = Uc + ((s * 4 + mu) * 9 + k) * 2;
      b[lk_off<S, NE>(k, lane)] = pack_from_double<S>(src[0], src[1], 0);
    }
  }
}

// Largest |row2 - conj(row0 x row1)| over the links of each block's sites
// (FP64, canonical layout): zero up to rounding exactly when every link is
// in SU(3), so that row 2 need not be stored.
__global__ __launch_bounds__(256) void k_link_su3_dev(Geom g, const double* __restrict__ Uc,
                                                      double* __restrict__ partials) {
  SiteId id = site_id(g);
  double m = 0.0;
  if (id.valid) {
    const int64_t s = lex_site(g, id.par, id.h);
    for (int mu = 0; mu < 4; mu++) {
      const double* u = Uc + (s * 4 + mu) * 18;
      cx<double> e[9];
      for (int k = 0; k < 9; k++) e[k] = cx<double>(u[2 * k], u[2 * k + 1]);
      cx<double> r[9];
      for (int k = 0; k < 6; k++) r[k] = e[k];
      su3_third_row(r);
      for (int k = 6; k < 9; k++) {
        const double dr = r[k].re - e[k].re, di = r[k].im - e[k].im;
        m = fmax(m, sqrt(dr * dr + di * di));
      }
      if (!(m == m)) m = INFINITY;  // NaN input: not SU(3)
    }
  }
  __shared__ double red[4];
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void k_max_finish(const double* __restrict__ partials, int nrows, double* __restrict__ out) {
  __shared__ double red[16];
  double m = 0.0;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) m = fmax(m, partials[r]);
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = fmax(m, red[w]);
    *out = fmax(red[0], m);
  }
}

// Canonical <-> native spinors, one thread per half index h: the sites
// (2j, y, z, t) and (2j + 1, y, z, t), 24 consecutive canonical complex numbers,
// are site h of parities p0 = (y + z + t) & 1 and p0 ^ 1, so a wave reads or
// writes one contiguous canonical segment and the field is streamed once.
// Geometry: the full lattice.  With `odd` set the native side is split by
// parity: even sites in dst, odd sites in odd, each a one-parity field.
__device__ __forceinline__ int64_t pair_site(const Geom& g, int h, int* p0) {
  const Coord c = decode(g, 0, h);
  *p0 = (c.y + c.z + c.t) & 1;
  return (c.x & ~1) + (int64_t)g.L[0] * (c.y + (int64_t)g.L[1] * (c.z + (int64_t)g.L[2] * c.t));
}

// dst = scale * src rounded to S (FP16 flushing to zero with ftz); |dst|^2
// partials per block (blocks past the half sites add zero rows, so a launch
// keeps site_grid(g) rows).
template <typename S>
__global__ __launch_bounds__(256) void k_pack_spinor(Geom g, S* __restrict__ dst, const double* __restrict__ src,
                                                     double scale, int ftz, double* __restrict__ partials,
                                                     S* __restrict__ odd) {
  using T = typename Traits<S>::T;
  const int h = blockIdx.x * 256 + threadIdx.x;
  const int rhs = blockIdx.y;
  src += (size_t)rhs * volume(g) * 24;
  double red[1] = {0.0};
  if (h < g.Vh) {
    int p0;
    const int64_t s0 = pair_site(g, h, &p0);
    const double2* s2 = reinterpret_cast<const double2*>(src) + s0 * 12;  // one 16-byte load per complex
    const int lane = h & 63;
    T acc = 0;
    for (int q = 0; q < 2; q++) {
      const int par = p0 ^ q;
      S* b = odd ? (par ? odd : dst) + (size_t)rhs * g.nb * 768 + sp_block(g, 0, h)
                 : dst + (size_t)rhs * spinor_elems(g) + sp_block(g, par, h);
      for (int k = 0; k < 12; k++) {
        const double2 c = s2[q * 12 + k];
        const S v = pack_from_double<S>(scale * c.x, scale * c.y, ftz);
        b[sp_off<S>(k, lane)] = v;
        acc += norm2(Traits<S>::load(&v));
      }
    }
    red[0] = acc;
  }
  if (partials) block_reduce_store<1>(red, partials + (size_t)rhs * gridDim.x, blockIdx.x);
}

// canon = scale * double(src) with scale = scale_dev[rhs] (if given) or scale.
template <typename S>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geom g, double* __restrict__ dst, const S* __restrict__ src,
                                                       const double* __restrict__ scale_dev, double scale,
                                                       const S* __restrict__ odd) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const int rhs = blockIdx.y;
  dst += (size_t)rhs * volume(g) * 24;
  if (scale_dev) scale = scale_dev[rhs];
  int p0;
  const int64_t s0 = pair_site(g, h, &p0);
  double2* d2 = reinterpret_cast<double2*>(dst) + s0 * 12;  // one 16-byte store per complex
  for (int q = 0; q < 2; q++) {
    const int par = p0 ^ q;
    cx<typename Traits<S>::T> f[12];
    if (odd)
      load_site((par ? odd : src) + (size_t)rhs * g.nb * 768, g, 0, h, f);
    else
      load_site(src + (size_t)rhs * spinor_elems(g), g, par, h, f);
    for (int k = 0; k < 12; k++) d2[q * 12 + k] = make_double2(scale * (double)f[k].re, scale * (double)f[k].im);
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_zero(Geom g, S* __restrict__ dst) {
  using Gr = typename Lay<S>::Gran;
  const size_t n = spinor_granules<S>(g);
  dst += (size_t)blockIdx.y * spinor_elems(g);
  Gr z;
  for (int c = 0; c < Lay<S>::C; c++) z.s[c] = Traits<S>::pack(cx<typename Traits<S>::T>(0, 0), 0);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
    reinterpret_cast<Gr*>(dst)[e] = z;
}

// dst = src for the one-parity fields of blockIdx.y right-hand sides, whose
// vectors start dst_stride / src_stride elements apart: the even half of a full
// field has the one-parity layout at the field's start, so this moves even-odd
// vectors into and out of full fields.
template <typename S>
__global__ __launch_bounds__(256) void k_copy_fields(Geom gh, S* __restrict__ dst, size_t dst_stride,
                                                     const S* __restrict__ src, size_t src_stride) {
  using Gr = typename Lay<S>::Gran;
  const size_t n = spinor_granules<S>(gh);
  Gr* d = reinterpret_cast<Gr*>(dst + (size_t)blockIdx.y * dst_stride);
  const Gr* a = reinterpret_cast<const Gr*>(src + (size_t)blockIdx.y * src_stride);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) d[e] = a[e];
}

// ---------------------------------------------------------------------------
// BiCGStab body (Alg. 4 / Alg. 5).  Vectors: x, r (holds s between the two
// matrix applications), r*, p, v, t.  All are walked granule by granule.

#define QCD_FLAT_LOOP(S) \
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x, n_ = spinor_granules<S>(g); e < n_; \
       e += (size_t)gridDim.x * 256)
#define QCD_RHS_OFFSET(S, ptr) ptr += (size_t)blockIdx.y * spinor_elems(g)

template <typename S> using GrOf = typename Lay<S>::Gran;

// p := beta (p - omega' v) + r, with the previous iteration's rescaling of
// p and v by gamma folded into the coefficient (pcoef = beta * gamma).  In
// the first iteration p = r (p = v = 0 initially).
template <typename S>
__global__ __launch_bounds__(256) void k_p_update(Geom g, const Scalars* __restrict__ scal, S* __restrict__ p,
                                                  const S* __restrict__ v, const S* __restrict__ r, int ftz) {
  using T = typename Traits<S>::T;
  using Gr = GrOf<S>;
  const Scalars* sc = scal + blockIdx.y;
  if (!sc->active) return;
  QCD_RHS_OFFSET(S, p); QCD_RHS_OFFSET(S, v); QCD_RHS_OFFSET(S, r);
  const int first = sc->first;
  const cx<T> c((T)sc->pcoef[0], (T)sc->pcoef[1]);
  const cx<T> w((T)sc->omega_prev[0], (T)sc->omega_prev[1]);
  QCD_FLAT_LOOP(S) {
    if (!gran_valid<S>(g, e)) continue;
    const Gr rg = reinterpret_cast<const Gr*>(r)[e];
    Gr out;
    if (first) {
      out = rg;
    } else {
      const Gr pg = reinterpret_cast<const Gr*>(p)[e];
      const Gr vg = reinterpret_cast<const Gr*>(v)[e];
#pragma unroll
      for (int i = 0; i < Lay<S>::C; i++) {
        const cx<T> o = c * (Traits<S>::load(&pg.s[i]) - w * Traits<S>::load(&vg.s[i])) + Traits<S>::load(&rg.s[i]);
        out.s[i] = Traits<S>::pack(o, ftz);
      }
    }
    reinterpret_cast<Gr*>(p)[e] = out;
  }
}

// r := r - alpha v   (the vector s of the standard formulation)
template <typename S>
__global__ __launch_bounds__(256) void k_s_update(Geom g, const Scalars* __restrict__ scal, S* __restrict__ r,
                                                  const S* __restrict__ v, int ftz) {
  using T = typename Traits<S>::T;
  using Gr = GrOf<S>;
  const Scalars* sc = scal + blockIdx.y;
  if (!sc->active) return;
  QCD_RHS_OFFSET(S, r); QCD_RHS_OFFSET(S, v);
  const cx<T> a((T)sc->alpha[0], (T)sc->alpha[1]);
  QCD_FLAT_LOOP(S) {
    if (!gran_valid<S>(g, e)) continue;
    Gr rg = reinterpret_cast<const Gr*>(r)[e];
    const Gr vg = reinterpret_cast<const Gr*>(v)[e];
#pragma unroll
    for (int i = 0; i < Lay<S>::C; i++)
      rg.s[i] = Traits<S>::pack(Traits<S>::load(&rg.s[i]) - a * Traits<S>::load(&vg.s[i]), ftz);
    reinterpret_cast<Gr*>(r)[e] = rg;
  }
}

// x := xscale x + (lambda'/gamma') (omega s + alpha p);
// r := gamma_pred (s - omega t), stored in the buffer that held s.
// Partials: |s - omega t|^2 before the rescaling (unrounded), and from the
// stored values |r|^2, (r*, r) and |x|^2.  Each thread accumulates in the
// arithmetic precision, the block and the finish kernel in FP64.
template <typename S>
__global__ __launch_bounds__(256) void k_xr_update(Geom g, const Scalars* __restrict__ scal, S* __restrict__ x,
                                                   S* __restrict__ r, const S* __restrict__ t,
                                                   const S* __restrict__ p, const S* __restrict__ rstar,
                                                   double* __restrict__ partials, int ftz) {
  using T = typename Traits<S>::T;
  using Gr = GrOf<S>;
  const Scalars* sc = scal + blockIdx.y;
  if (!sc->active) return;
  QCD_RHS_OFFSET(S, x); QCD_RHS_OFFSET(S, r); QCD_RHS_OFFSET(S, t); QCD_RHS_OFFSET(S, p); QCD_RHS_OFFSET(S, rstar);
  const int first = sc->first;
  const T xs = (T)sc->xscale, xc = (T)sc->xcoef, gp = (T)sc->gamma_pred;
  const cx<T> om((T)sc->omega[0], (T)sc->omega[1]);
  const cx<T> al((T)sc->alpha[0], (T)sc->alpha[1]);
  T ww = 0, rr = 0, rsr_re = 0, rsr_im = 0, xx = 0;
  QCD_FLAT_LOOP(S) {
    if (!gran_valid<S>(g, e)) continue;
    const Gr sg = reinterpret_cast<const Gr*>(r)[e];
    const Gr pg = reinterpret_cast<const Gr*>(p)[e];
    const Gr tg = reinterpret_cast<const Gr*>(t)[e];
    const Gr qg = reinterpret_cast<const Gr*>(rstar)[e];
    Gr xg;
    if (!first) xg = reinterpret_cast<const Gr*>(x)[e];
    Gr xo, ro;
#pragma unroll
    for (int i = 0; i < Lay<S>::C; i++) {
      const cx<T> s = Traits<S>::load(&sg.s[i]);
      cx<T> xn = xc * (om * s + al * Traits<S>::load(&pg.s[i]));
      if (!first) xn = xs * Traits<S>::load(&xg.s[i]) + xn;
      xo.s[i] = Traits<S>::pack(xn, ftz);
      const cx<T> w = s - om * Traits<S>::load(&tg.s[i]);
      ro.s[i] = Traits<S>::pack(gp * w, ftz);
      const cx<T> rs = Traits<S>::load(&ro.s[i]), xsv = Traits<S>::load(&xo.s[i]);
      const cx<T> q = Traits<S>::load(&qg.s[i]);
      ww += norm2(w);
      rr += norm2(rs);
      rsr_re += q.re * rs.re + q.im * rs.im;
      rsr_im += q.re * rs.im - q.im * rs.re;
      xx += norm2(xsv);
    }
    reinterpret_cast<Gr*>(x)[e] = xo;
    reinterpret_cast<Gr*>(r)[e] = ro;
  }
  double red[5] = {(double)ww, (double)rr, (double)rsr_re, (double)rsr_im, (double)xx};
  block_reduce_store<5>(red, partials + (size_t)blockIdx.y * gridDim.x * 5, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Refinement step (Alg. 3): y~ = low(scale * r) with scale = s / |r|;
// the inner solver starts from r = r* = y~.  Partials: sum single(y~)^2 in
// the arithmetic precision per site (FP64 across sites), and the number of
// zero reals in y~ (the underflow diagnostic of Fig. 9).
template <typename S>
__global__ __launch_bounds__(256) void k_convert(Geom g, const Scalars* __restrict__ scal,
                                                 const double2* __restrict__ r64, S* __restrict__ y,
                                                 S* __restrict__ rstar, double* __restrict__ partials, int ftz) {
  using T = typename Traits<S>::T;
  using Gr = GrOf<S>;
  constexpr int C = Lay<S>::C;
  const Scalars* sc = scal + blockIdx.y;
  if (!sc->outer_active || (sc->dev_outer && !sc->outer_step)) return;
  SiteId id = site_id(g);
  r64 += (size_t)blockIdx.y * spinor_elems(g);
  QCD_RHS_OFFSET(S, y); QCD_RHS_OFFSET(S, rstar);
  double red[2] = {0, 0};
  if (id.valid) {
    const double sc_ = sc->out_scale;
    cx<double> f[12];
    load_site(r64, g, id.par, id.h, f);
    S* yb = y + sp_block(g, id.par, id.h) + (id.h & 63) * C;
    S* qb = rstar + sp_block(g, id.par, id.h) + (id.h & 63) * C;
    T acc = 0;
    int zeros = 0;
#pragma unroll
    for (int j = 0; j < Lay<S>::G; j++) {
      Gr v;
#pragma unroll
      for (int c = 0; c < C; c++) {
        const int k = j * C + c;
        v.s[c] = pack_from_double<S>(sc_ * f[k].re, sc_ * f[k].im, ftz);
        const cx<T> q = Traits<S>::load(&v.s[c]);
        acc += norm2(q);
        zeros += (q.re == (T)0) + (q.im == (T)0);
      }
      *reinterpret_cast<Gr*>(yb + j * 64 * C) = v;
      *reinterpret_cast<Gr*>(qb + j * 64 * C) = v;
    }
    red[0] = acc;
    red[1] = zeros;
  }
  block_reduce_store<2>(red, partials + (size_t)blockIdx.y * gridDim.x * 2, blockIdx.x);
}

// x64 := x64 + (|r| / s^) * double(x_inner), with x_inner = xscale * X / lambda'
// (skipped for right-hand sides whose inner solve made no step).
template <typename S>
__global__ __launch_bounds__(256) void k_correct(Geom g, const Scalars* __restrict__ scal, double2* __restrict__ x64,
                                                 const S* __restrict__ xlo) {
  const Scalars* sc = scal + blockIdx.y;
  if (!sc->outer_active || sc->iter == 0 || sc->status == kNonFinite) return;
  if (sc->dev_outer && !sc->outer_step) return;
  SiteId id = site_id(g);
  if (!id.valid) return;
  x64 += (size_t)blockIdx.y * spinor_elems(g);
  QCD_RHS_OFFSET(S, xlo);
  const double c = sc->out_rnorm / sc->shat * sc->xscale / sc->lambda_cum;
  cx<typename Traits<S>::T> f[12];
  cx<double> xo[12];
  load_site(xlo, g, id.par, id.h, f);
  load_site(x64, g, id.par, id.h, xo);
  for (int k = 0; k < 12; k++) {
    xo[k].re += c * (double)f[k].re;
    xo[k].im += c * (double)f[k].im;
  }
  store_site(x64, g, id.par, id.h, xo, 0);
}

// The end of an even-odd solve in one pass: x_o = eta_o + kappa t with t =
// H_oe x_e from the last refinement step's hop (eq. (6)), and the canonical
// solution (x_e from its one-parity field, x_o as formed) written pair by pair
// as in k_unpack_spinor, so x_o never goes through memory; the odd rows
// eta_o - (x_o - kappa t) of b - D x as |.|^2 partials per block of half sites
// (site_grid of the one-parity geometry).  g: the full lattice; one-parity FP64
// fields; right-hand side blockIdx.y.
__global__ __launch_bounds__(256) void k_eo_recon_unpack(Geom g, double* __restrict__ canon,
                                                         const double2* __restrict__ xe,
                                                         const double2* __restrict__ eta,
                                                         const double2* __restrict__ t, double kappa,
                                                         double* __restrict__ partials) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  const int rhs = blockIdx.y;
  double red[1] = {0.0};
  if (h < g.Vh) {
    const size_t o = (size_t)rhs * g.nb * 768;  // one-parity field of this right-hand side
    int p0;
    const int64_t s0 = pair_site(g, h, &p0);
    double2* d2 = reinterpret_cast<double2*>(canon + (size_t)rhs * volume(g) * 24) + s0 * 12;
    // the pair's even site goes to slot p0, its odd site to slot 1 - p0: the
    // same instructions for every lane, only the store addresses differ
    cx<double> x[12];
    load_site(xe + o, g, 0, h, x);
    for (int k = 0; k < 12; k++) d2[p0 * 12 + k] = make_double2(x[k].re, x[k].im);
    cx<double> e[12], tt[12];
    load_site(eta + o, g, 0, h, e);
    load_site(t + o, g, 0, h, tt);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 12; k++) {
      x[k] = cx<double>(e[k].re + kappa * tt[k].re, e[k].im + kappa * tt[k].im);
      const double rr = e[k].re - (x[k].re - kappa * tt[k].re), ri = e[k].im - (x[k].im - kappa * tt[k].im);
      acc += rr * rr + ri * ri;
    }
    for (int k = 0; k < 12; k++) d2[(1 - p0) * 12 + k] = make_double2(x[k].re, x[k].im);
    red[0] = acc;
  }
  block_reduce_store<1>(red, partials + (size_t)rhs * gridDim.x, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Finish kernels: block b sums the partial rows of right-hand side b, thread
// 0 updates that right-hand side's scalars.

__device__ __forceinline__ cx<double> cd(const double* a) { return cx<double>(a[0], a[1]); }
__device__ __forceinline__ void setc(double* a, cx<double> v) { a[0] = v.re; a[1] = v.im; }
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return cx<double>((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__device__ __forceinline__ bool finite_c(cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

// End of an inner solve; with device-driven refinement its refinement step becomes due.
__device__ void stop(Scalars* sc, int status) {
  sc->status = status;
  sc->active = 0;
  if (sc->dev_outer && sc->outer_active) sc->outer_step = 1;
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

#define QCD_FINISH_BEGIN(NV)                                                  \
  Scalars* sc = scal + blockIdx.x;                                            \
  double s[NV];                                                               \
  finish_sum<NV>(partials + (size_t)blockIdx.x * nrows * NV, nrows, s);       \
  if (threadIdx.x != 0) return;

__global__ void k_bicg_init(Scalars* scal, const double* partials, int nrows) {
  QCD_FINISH_BEGIN(1)
  bicg_init_dev(sc, s[0]);
}

// alpha = rho / (r*, v)
__global__ void k_alpha(Scalars* scal, const double* partials, int nrows) {
  if (!scal[blockIdx.x].active) return;
  QCD_FINISH_BEGIN(2)
  const cx<double> rv(s[0], s[1]);
  if (rv.re == 0.0 && rv.im == 0.0) { stop(sc, kBreakdown); return; }
  const cx<double> a = cdiv(cd(sc->rho), rv);
  if (!finite_c(a)) { stop(sc, kNonFinite); return; }
  setc(sc->alpha, a);
}

// omega = (t,s)/(t,t) with the omega_0 prescription; the x-update factor
// lambda'/gamma'; and the factor that rescales the new residual to norm
// sigma, from |s - omega t|^2 = (s,s) - 2 Re(conj(omega)(t,s)) + |omega|^2 (t,t).
__global__ void k_omega(Scalars* scal, const double* partials, int nrows) {
  if (!scal[blockIdx.x].active) return;
  QCD_FINISH_BEGIN(4)
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
__global__ void k_iter_end(Scalars* scal, const double* partials, int nrows, double* history, int hist_stride) {
  if (!scal[blockIdx.x].active) return;
  QCD_FINISH_BEGIN(5)
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
  if (history && sc->iter < sc->max_iter) history[(size_t)blockIdx.x * hist_stride + sc->iter] = res2;
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

// Outer step: |r| of the FP64 residual, the rescaling factor s / |r| and the
// outer stopping test (|r| <= tol |b|); the first call (from the packing of
// b) also records |b|.
//
// Device-driven refinement (dev_outer): only right-hand sides whose step is
// due take part; the step is counted, the inner solve's iterations and stop
// reason are recorded, (|r|, zeros of the y~ this step solved with) is
// logged, and refining ends on a failed inner solve (non-finite, or no
// iteration: breakdown), a non-finite |r|, the tolerance or max_outer steps.
__global__ void k_outer_norm(Scalars* scal, const double* partials, int nrows, double s_target, double* log) {
  if (!scal[blockIdx.x].outer_active) return;
  if (scal[blockIdx.x].dev_outer && !scal[blockIdx.x].outer_step) return;
  QCD_FINISH_BEGIN(1)
  sc->out_rnorm = sqrt(s[0]);
  if (sc->out_bnorm < 0.0) sc->out_bnorm = sc->out_rnorm;
  sc->out_scale = (s[0] > 0.0) ? s_target / sc->out_rnorm : 0.0;
  if (sc->dev_outer) {
    const int k = sc->outer_count;
    if (log && k < kOuterLog) {
      log[((size_t)blockIdx.x * kOuterLog + k) * 2] = sc->out_rnorm;
      log[((size_t)blockIdx.x * kOuterLog + k) * 2 + 1] = sc->zeros;
    }
    sc->outer_count = k + 1;
    sc->inner_total += sc->iter;
    sc->last_status = sc->status;
    if (sc->status == kNonFinite || sc->iter == 0) {
      sc->fail = sc->status == kNonFinite ? kNonFinite : kBreakdown;
      sc->outer_active = 0;
      return;
    }
    if (!isfinite(sc->out_rnorm)) {
      sc->fail = kNonFinite;
      sc->outer_active = 0;
      return;
    }
  }
  if (!(sc->out_rnorm > sc->out_tol * sc->out_bnorm)) sc->outer_active = 0;
  if (sc->dev_outer && sc->outer_count >= sc->max_outer) sc->outer_active = 0;
}

// Start of the device-driven refinement, after the start norm |b'| (k_outer_norm):
// |b| of the full system (b2: |b|^2 of the even-odd form's b, else |b'| = |b|),
// the even-odd stop test taken relative to it, and the step bookkeeping.
__global__ void k_ir_dev_start(Scalars* scal, const double* b2, double tol, int max_outer) {
  if (threadIdx.x != 0) return;
  Scalars* sc = scal + blockIdx.x;
  if (b2) {
    const double bf = sqrt(b2[blockIdx.x]), bp = sc->out_rnorm;
    sc->bfull = bf;
    if (bp > 0 && isfinite(bp)) sc->out_tol = tol * bf / bp;
  } else {
    sc->bfull = sc->out_rnorm;
  }
  sc->dev_outer = 1;
  sc->outer_step = sc->outer_active ? 1 : 0;
  sc->max_outer = max_outer;
  sc->outer_count = sc->inner_total = sc->fail = 0;
  sc->last_status = kConverged;
  sc->first_shat = 0.0;
}

// After the conversion: s^ (Alg. 3) and the start of the inner BiCGStab.
// Device-driven refinement: only a right-hand side whose step is due
// continues (the flag is cleared before the inner start, which raises it
// again if that start stops at once, so the next step sees it).
__global__ void k_convert_finish(Scalars* scal, const double* partials, int nrows, int recalc_shat, double s_target) {
  if (scal[blockIdx.x].dev_outer && !scal[blockIdx.x].outer_step) return;
  if (!scal[blockIdx.x].outer_active) {
    if (threadIdx.x == 0) {
      scal[blockIdx.x].active = 0;
      scal[blockIdx.x].iter = 0;
      scal[blockIdx.x].outer_step = 0;
    }
    return;
  }
  QCD_FINISH_BEGIN(2)
  sc->shat = recalc_shat ? sqrt(s[0]) : s_target;
  sc->zeros = s[1];
  if (sc->outer_count == 0) sc->first_shat = sc->shat;
  sc->outer_step = 0;
  bicg_init_dev(sc, s[0]);
}

__global__ void k_finish_sum_any(const double* partials, int nrows, int nv, double* out) {
  // generic: sums up to 8 columns of right-hand side blockIdx.x
  partials += (size_t)blockIdx.x * nrows * nv;
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
      out[(size_t)blockIdx.x * nv + i] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 native -> storage precision (one RNE conversion), with |stored|^2
// partials per block; and storage precision -> FP64 times a per-RHS scale.
template <typename S>
__global__ __launch_bounds__(256) void k_narrow(Geom g, S* __restrict__ dst, const double2* __restrict__ src,
                                                double* __restrict__ partials, int ftz) {
  using T = typename Traits<S>::T;
  SiteId id = site_id(g);
  const int rhs = blockIdx.y;
  dst += (size_t)rhs * spinor_elems(g);
  src += (size_t)rhs * spinor_elems(g);
  double red[1] = {0.0};
  if (id.valid) {
    cx<double> f[12];
    load_site(src, g, id.par, id.h, f);
    S* b = dst + sp_block(g, id.par, id.h);
    const int lane = id.h & 63;
    T acc = 0;
    for (int k = 0; k < 12; k++) {
      const S v = pack_from_double<S>(f[k].re, f[k].im, ftz);
      b[sp_off<S>(k, lane)] = v;
      acc += norm2(Traits<S>::load(&v));
    }
    red[0] = acc;
  }
  if (partials) block_reduce_store<1>(red, partials + (size_t)rhs * gridDim.x, blockIdx.x);
}

template <typename S>
__global__ __launch_bounds__(256) void k_widen(Geom g, double2* __restrict__ dst, const S* __restrict__ src,
                                               const double* __restrict__ scale_dev) {
  SiteId id = site_id(g);
  if (!id.valid) return;
  const int rhs = blockIdx.y;
  dst += (size_t)rhs * spinor_elems(g);
  src += (size_t)rhs * spinor_elems(g);
  const double c = scale_dev[rhs];
  cx<typename Traits<S>::T> f[12];
  cx<double> o[12];
  load_site(src, g, id.par, id.h, f);
  for (int k = 0; k < 12; k++) o[k] = cx<double>(c * (double)f[k].re, c * (double)f[k].im);
  store_site(dst, g, id.par, id.h, o, 0);
}

// launchers

#define QCD_DISPATCH(prec, FN, ...)                     \
  do {                                                  \
    if ((prec) == kFP64) FN<double2>(__VA_ARGS__);      \
    else if ((prec) == kFP32) FN<float2>(__VA_ARGS__);  \
    else if ((prec) == kBF16) FN<bf2>(__VA_ARGS__);     \
    else FN<__half2>(__VA_ARGS__);                      \
  } while (0)

template <typename S> static void pack_links_t(const Geom& g, void* dst, const double* U, int recon, hipStream_t st) {
  if (recon)
    hipLaunchKernelGGL((k_pack_links<S, 6>), dim3(site_grid(g)), dim3(256), 0, st, g, (S*)dst, U);
  else
    hipLaunchKernelGGL((k_pack_links<S, 9>), dim3(site_grid(g)), dim3(256), 0, st, g, (S*)dst, U);
}
void launch_pack_links(const Geom& g, int prec, void* dst, const double* U, int recon, hipStream_t st) {
  QCD_DISPATCH(prec, pack_links_t, g, dst, U, recon, st);
}
void launch_link_su3_dev(const Geom& g, const double* U, double* partials, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_link_su3_dev, dim3(site_grid(g)), dim3(256), 0, st, g, U, partials);
  hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(1024), 0, st, (const double*)partials, site_grid(g), out);
}

template <typename S>
static void pack_spinor_t(const Geom& g, int n, void* dst, const double* c, double scale, int ftz, double* partials,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_pack_spinor<S>, dim3(site_grid(g), n), dim3(256), 0, st, g, (S*)dst, c, scale, ftz, partials,
                     nullptr);
}
void launch_pack_spinor(const Geom& g, int prec, int n, void* dst, const double* canon, double scale, int ftz,
                        double* partials, hipStream_t st) {
  QCD_DISPATCH(prec, pack_spinor_t, g, n, dst, canon, scale, ftz, partials, st);
}

template <typename S>
static void unpack_spinor_t(const Geom& g, int n, double* c, const void* src, const double* sd, double scale,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_spinor<S>, dim3((g.Vh + 255) / 256, n), dim3(256), 0, st, g, c, (const S*)src, sd,
                     scale, nullptr);
}
void launch_unpack_spinor(const Geom& g, int prec, int n, double* canon, const void* src, const double* scale_dev,
                          double scale, hipStream_t st) {
  QCD_DISPATCH(prec, unpack_spinor_t, g, n, canon, src, scale_dev, scale, st);
}

void launch_pack_spinor_split(const Geom& g, int n, void* even, void* odd, const double* canon, double* partials,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_pack_spinor<double2>, dim3(site_grid(g), n), dim3(256), 0, st, g, (double2*)even, canon, 1.0,
                     0, partials, (double2*)odd);
}
void launch_unpack_spinor_split(const Geom& g, int n, double* canon, const void* even, const void* odd,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_spinor<double2>, dim3((g.Vh + 255) / 256, n), dim3(256), 0, st, g, canon,
                     (const double2*)even, nullptr, 1.0, (const double2*)odd);
}

// Complex normal values z = (g0 + i g1) / sqrt(2) (so E|z|^2 = 1) in
// canonical complex128 order: component j takes draws 2j and 2j + 1 of a
// counter-based SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014: the
// draw n of the stream with key k is the SplitMix64 finaliser of
// k + (n + 1) * golden gamma, key = finaliser(seed + gamma)), mapped to (0, 1]
// with 53 bits and paired by the Box-Muller transform.  Values depend only on
// (seed, j), not on the launch shape.
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
constexpr uint64_t kSm64Gamma = 0x9e3779b97f4a7c15ULL;
__device__ __forceinline__ double sm64_unit(uint64_t key, uint64_t n) {
  return (double)((sm64_mix(key + (n + 1) * kSm64Gamma) >> 11) + 1) * (1.0 / 9007199254740992.0);
}
__global__ __launch_bounds__(256) void k_gaussian(double2* __restrict__ out, int64_t n, uint64_t key) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const double u1 = sm64_unit(key, 2 * (uint64_t)j), u2 = sm64_unit(key, 2 * (uint64_t)j + 1);
    const double r = sqrt(-2.0 * log(u1)) * 0.70710678118654752440;
    double sn, cs;
    sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
    out[j] = make_double2(r * cs, r * sn);
  }
}
void launch_gaussian(double* out, int64_t ncomplex, uint64_t seed, hipStream_t st) {
  const uint64_t key = sm64_mix(seed + kSm64Gamma);
  const int64_t blocks = std::min<int64_t>((ncomplex + 255) / 256, 65536);
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, (double2*)out,
                     ncomplex, key);
}

template <typename S> static void zero_t(const Geom& g, int n, void* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<S>, dim3(flat_grid<S>(g), n), dim3(256), 0, st, g, (S*)dst);
}
void launch_zero(const Geom& g, int prec, int n, void* dst, hipStream_t st) {
  QCD_DISPATCH(prec, zero_t, g, n, dst, st);
}
template <typename S>
static void copy_fields_t(const Geom& gh, int n, void* dst, size_t dst_stride, const void* src, size_t src_stride,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_copy_fields<S>, dim3(flat_grid<S>(gh), n), dim3(256), 0, st, gh, (S*)dst, dst_stride,
                     (const S*)src, src_stride);
}
void launch_copy_fields(const Geom& gh, int prec, int n, void* dst, size_t dst_stride, const void* src,
                        size_t src_stride, hipStream_t st) {
  QCD_DISPATCH(prec, copy_fields_t, gh, n, dst, dst_stride, src, src_stride, st);
}

void launch_bicg_init(int n, Scalars* sc, const double* partials, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_bicg_init, dim3(n), dim3(1024), 0, st, sc, partials, nrows);
}

template <typename S>
static void p_update_t(const Geom& g, int n, Scalars* sc, void* p, const void* v, const void* r, int ftz,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_p_update<S>, dim3(flat_grid<S>(g), n), dim3(256), 0, st, g, sc, (S*)p, (const S*)v,
                     (const S*)r, ftz);
}
void launch_p_update(const Geom& g, int prec, int n, Scalars* sc, void* p, const void* v, const void* r, int ftz,
                     hipStream_t st) {
  QCD_DISPATCH(prec, p_update_t, g, n, sc, p, v, r, ftz, st);
}

void launch_alpha(int n, Scalars* sc, const double* partials, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_alpha, dim3(n), dim3(1024), 0, st, sc, partials, nrows);
}

template <typename S>
static void s_update_t(const Geom& g, int n, Scalars* sc, void* r, const void* v, int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_s_update<S>, dim3(flat_grid<S>(g), n), dim3(256), 0, st, g, sc, (S*)r, (const S*)v, ftz);
}
void launch_s_update(const Geom& g, int prec, int n, Scalars* sc, void* r, const void* v, int ftz, hipStream_t st) {
  QCD_DISPATCH(prec, s_update_t, g, n, sc, r, v, ftz, st);
}

void launch_omega(int n, Scalars* sc, const double* partials, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_omega, dim3(n), dim3(1024), 0, st, sc, partials, nrows);
}

template <typename S>
static void xr_update_t(const Geom& g, int n, Scalars* sc, void* x, void* r, const void* t, const void* p,
                        const void* rs, double* partials, int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_xr_update<S>, dim3(flat_grid<S>(g), n), dim3(256), 0, st, g, sc, (S*)x, (S*)r, (const S*)t,
                     (const S*)p, (const S*)rs, partials, ftz);
}
void launch_xr_update(const Geom& g, int prec, int n, Scalars* sc, void* x, void* r, const void* t, const void* p,
                      const void* rstar, double* partials, int ftz, hipStream_t st) {
  QCD_DISPATCH(prec, xr_update_t, g, n, sc, x, r, t, p, rstar, partials, ftz, st);
}

void launch_iter_end(int n, Scalars* sc, const double* partials, int nrows, double* history, int hist_stride,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_iter_end, dim3(n), dim3(1024), 0, st, sc, partials, nrows, history, hist_stride);
}

void launch_outer_residual_norm(int n, Scalars* sc, const double* partials, int nrows, double s_target,
                                hipStream_t st, double* log) {
  hipLaunchKernelGGL(k_outer_norm, dim3(n), dim3(1024), 0, st, sc, partials, nrows, s_target, log);
}

template <typename S>
static void convert_t(const Geom& g, int n, Scalars* sc, const double* r64, void* y, void* rstar, double* partials,
                      int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_convert<S>, dim3(site_grid(g), n), dim3(256), 0, st, g, sc, (const double2*)r64, (S*)y,
                     (S*)rstar, partials, ftz);
}
void launch_convert(const Geom& g, int prec, int n, Scalars* sc, const double* r64, void* y, void* rstar,
                    double* partials, int ftz, hipStream_t st) {
  QCD_DISPATCH(prec, convert_t, g, n, sc, r64, y, rstar, partials, ftz, st);
}

void launch_ir_dev_start(int n, Scalars* sc, const double* b2_dev, double tol, int max_outer, hipStream_t st) {
  hipLaunchKernelGGL(k_ir_dev_start, dim3(n), dim3(64), 0, st, sc, b2_dev, tol, max_outer);
}
void launch_convert_finish(int n, Scalars* sc, const double* partials, int nrows, int recalc_shat, double s_target,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_convert_finish, dim3(n), dim3(1024), 0, st, sc, partials, nrows, recalc_shat, s_target);
}

template <typename S>
static void correct_t(const Geom& g, int n, Scalars* sc, double* x64, const void* xlo, hipStream_t st) {
  hipLaunchKernelGGL(k_correct<S>, dim3(site_grid(g), n), dim3(256), 0, st, g, sc, (double2*)x64, (const S*)xlo);
}
void launch_correct(const Geom& g, int prec, int n, Scalars* sc, double* x64, const void* xlo, hipStream_t st) {
  QCD_DISPATCH(prec, correct_t, g, n, sc, x64, xlo, st);
}

void launch_eo_recon_unpack(const Geom& g, int n, double* canon, const double* xe, const double* eta_o,
                            const double* t, double kappa, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_eo_recon_unpack, dim3((g.Vh + 255) / 256, n), dim3(256), 0, st, g, canon, (const double2*)xe,
                     (const double2*)eta_o, (const double2*)t, kappa, partials);
}
void launch_finish_sum(int n, const double* partials, int nrows, int nv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_sum_any, dim3(n), dim3(1024), 0, st, partials, nrows, nv, out);
}

}  // namespace qcd

namespace qcd {
template <typename S>
static void narrow_t(const Geom& g, int n, void* dst, const double* src, double* partials, int ftz, hipStream_t st) {
  hipLaunchKernelGGL(k_narrow<S>, dim3(site_grid(g), n), dim3(256), 0, st, g, (S*)dst, (const double2*)src, partials,
                     ftz);
}
void launch_narrow(const Geom& g, int prec, int n, void* dst, const double* src, double* partials, int ftz,
                   hipStream_t st) {
  QCD_DISPATCH(prec, narrow_t, g, n, dst, src, partials, ftz, st);
}
template <typename S>
static void widen_t(const Geom& g, int n, double* dst, const void* src, const double* scale_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_widen<S>, dim3(site_grid(g), n), dim3(256), 0, st, g, (double2*)dst, (const S*)src,
                     scale_dev);
}
void launch_widen(const Geom& g, int prec, int n, double* dst, const void* src, const double* scale_dev,
                  hipStream_t st) {
  QCD_DISPATCH(prec, widen_t, g, n, dst, src, scale_dev, st);
}
}  // namespace qcd

// ---------------------------------------------------------------------------
// Streaming probes of the memory system: the bandwidth a plain sweep reaches
// on this GPU, the ceiling the Wilson operator's bandwidth is read against.
// Every lane moves 16-byte granules, four independent ones per loop trip, in
// a grid-stride sweep; loads and stores are non-temporal (each byte is
// touched once).
namespace qcd {
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Reads n granules; the XOR of what a lane read is stored only if it equals a
// fixed pattern (so the loads stay live without adding traffic); the store
// index stays below the grid's thread count, which launch_stream_probe keeps
// at most n.
__global__ __launch_bounds__(256) void k_stream_read(const u32x4* __restrict__ src, size_t n,
                                                     u32x4* __restrict__ sink) {
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (; i + 3 * stride < n; i += 4 * stride) {
    const u32x4 a = __builtin_nontemporal_load(src + i);
    const u32x4 b = __builtin_nontemporal_load(src + i + stride);
    const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
    const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
    acc ^= (a ^ b) ^ (c ^ d);
  }
  for (; i < n; i += stride) acc ^= __builtin_nontemporal_load(src + i);
  if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xf39cc060u && acc.w == 0x5cedc834u)
    sink[(size_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, size_t n,
                                                     u32x4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const u32x4 a = __builtin_nontemporal_load(src + i);
    const u32x4 b = __builtin_nontemporal_load(src + i + stride);
    const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
    const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
    __builtin_nontemporal_store(c, dst + i + 2 * stride);
    __builtin_nontemporal_store(d, dst + i + 3 * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(256) void k_stream_write(size_t n, u32x4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * 256;
  const u32x4 v = {(unsigned)blockIdx.x, (unsigned)threadIdx.x, 0u, 0u};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) __builtin_nontemporal_store(v, dst + i);
}

// mode 0: read src; 1: copy src -> dst; 2: write dst.  bytes a multiple of 16.
void launch_stream_probe(int mode, void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  // 8 blocks of 256 threads per compute unit (256 CUs), never more threads than granules
  const unsigned grid = (unsigned)std::max<size_t>(1, std::min<size_t>(2048, n / 256));
  if (mode == 0)
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, st, (const u32x4*)src, n, (u32x4*)dst);
  else if (mode == 1)
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, st, (const u32x4*)src, n, (u32x4*)dst);
  else
    hipLaunchKernelGGL(k_stream_write, dim3(grid), dim3(256), 0, st, n, (u32x4*)dst);
}
}  // namespace qcd
