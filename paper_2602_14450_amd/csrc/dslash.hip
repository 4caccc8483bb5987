// Wilson hopping stencil on the native layout.
//
// The Wilson matrix (eq. (1) of Kanamori et al., Sec. 2) is
//   D phi(x) = phi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) phi(x+mu)
//                                      + (1 + gamma_mu) U_mu(x-mu)^dag phi(x-mu) ].
// Each of the eight hops follows the three steps of Sec. 2: project the
// four-spinor to two colour vectors with (1 -/+ gamma_mu), multiply both by
// the SU(3) link (or its adjoint), and rebuild the four-spinor while
// accumulating.  The projection/reconstruction table below is derived for
// the Dirac basis whose gamma_1 is the matrix printed in Sec. 2:
//
//   (1 - g1): h1 = f1 + i f4, h2 = f2 + i f3;  rebuilt (h1, h2, -i h2, -i h1)
//   (1 + g1): h1 = f1 - i f4, h2 = f2 - i f3;  rebuilt (h1, h2,  i h2,  i h1)
//   (1 - g2): h1 = f1 + f4,   h2 = f2 - f3;    rebuilt (h1, h2,  -h2,   h1)
//   (1 + g2): h1 = f1 - f4,   h2 = f2 + f3;    rebuilt (h1, h2,   h2,  -h1)
//   (1 - g3): h1 = f1 + i f3, h2 = f2 - i f4;  rebuilt (h1, h2, -i h1,  i h2)
//   (1 + g3): h1 = f1 - i f3, h2 = f2 + i f4;  rebuilt (h1, h2,  i h1, -i h2)
//   (1 - g4): h1 = 2 f3,      h2 = 2 f4;       rebuilt (0, 0, h1, h2)
//   (1 + g4): h1 = 2 f1,      h2 = 2 f2;       rebuilt (h1, h2, 0, 0)
//
// D^dagger = gamma_5 D gamma_5 is the same stencil with gamma_mu -> -gamma_mu.
// One thread computes one output site; partial sums for the solver's dot
// products are formed from the values in registers (epilogues), so that the
// vectors they need are not read a second time.
#include "common.h"
#include "internal.h"

namespace qcd {

// Spin projection for direction MU; MINUS selects (1 - gamma_MU).
template <int MU, bool MINUS, typename T>
__device__ __forceinline__ void project(const cx<T> (&f)[4][3], cx<T> (&h1)[3], cx<T> (&h2)[3]) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    if constexpr (MU == 0) {
      h1[c] = MINUS ? f[0][c] + mul_i(f[3][c]) : f[0][c] - mul_i(f[3][c]);
      h2[c] = MINUS ? f[1][c] + mul_i(f[2][c]) : f[1][c] - mul_i(f[2][c]);
    } else if constexpr (MU == 1) {
      h1[c] = MINUS ? f[0][c] + f[3][c] : f[0][c] - f[3][c];
      h2[c] = MINUS ? f[1][c] - f[2][c] : f[1][c] + f[2][c];
    } else if constexpr (MU == 2) {
      h1[c] = MINUS ? f[0][c] + mul_i(f[2][c]) : f[0][c] - mul_i(f[2][c]);
      h2[c] = MINUS ? f[1][c] - mul_i(f[3][c]) : f[1][c] + mul_i(f[3][c]);
    } else {
      h1[c] = MINUS ? f[2][c] + f[2][c] : f[0][c] + f[0][c];
      h2[c] = MINUS ? f[3][c] + f[3][c] : f[1][c] + f[1][c];
    }
  }
}

// Reconstruct the four-spinor from the multiplied half-spinors and accumulate.
template <int MU, bool MINUS, typename T>
__device__ __forceinline__ void accumulate(cx<T> (&a)[4][3], const cx<T> (&u1)[3], const cx<T> (&u2)[3]) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    if constexpr (MU == 3) {
      if constexpr (MINUS) { a[2][c] = a[2][c] + u1[c]; a[3][c] = a[3][c] + u2[c]; }
      else { a[0][c] = a[0][c] + u1[c]; a[1][c] = a[1][c] + u2[c]; }
    } else {
      a[0][c] = a[0][c] + u1[c];
      a[1][c] = a[1][c] + u2[c];
      if constexpr (MU == 0) {
        if constexpr (MINUS) { a[2][c] = a[2][c] + mul_mi(u2[c]); a[3][c] = a[3][c] + mul_mi(u1[c]); }
        else { a[2][c] = a[2][c] + mul_i(u2[c]); a[3][c] = a[3][c] + mul_i(u1[c]); }
      } else if constexpr (MU == 1) {
        if constexpr (MINUS) { a[2][c] = a[2][c] - u2[c]; a[3][c] = a[3][c] + u1[c]; }
        else { a[2][c] = a[2][c] + u2[c]; a[3][c] = a[3][c] - u1[c]; }
      } else {
        if constexpr (MINUS) { a[2][c] = a[2][c] + mul_mi(u1[c]); a[3][c] = a[3][c] + mul_i(u2[c]); }
        else { a[2][c] = a[2][c] + mul_i(u1[c]); a[3][c] = a[3][c] + mul_mi(u2[c]); }
      }
    }
  }
}

// Load the spin components a hop in direction MU needs (all four, or two
// for the t direction where the projector keeps only one spin pair).
template <int MU, bool MINUS, typename S, typename T>
__device__ __forceinline__ void load_spinor(const Geom& g, const S* __restrict__ in, int par, int h,
                                            cx<T> (&f)[4][3]) {
#pragma unroll
  for (int s = 0; s < 4; s++) {
    const bool need = (MU != 3) || (MINUS ? s >= 2 : s < 2);
    if (need) {
#pragma unroll
      for (int c = 0; c < 3; c++) f[s][c] = Traits<S>::load(in + sp_index(g, par, h, 3 * s + c));
    }
  }
}

template <typename S, typename T>
__device__ __forceinline__ void load_link(const Geom& g, const S* __restrict__ U, int mu, int par, int h,
                                          cx<T> (&u)[9]) {
#pragma unroll
  for (int k = 0; k < 9; k++) u[k] = Traits<S>::load(U + lk_index(g, mu, par, h, k));
}

// One forward and one backward hop in direction MU.
template <int MU, bool DAG, typename S, typename T>
__device__ __forceinline__ void hop_dir(const Geom& g, const S* __restrict__ in, const S* __restrict__ U, int par,
                                        int h, const Coord& c, cx<T> (&a)[4][3]) {
  constexpr bool FWD_MINUS = !DAG;  // forward hop uses (1 - gamma) for D
  const int npar = par ^ 1;
  int hf, hb;
  if constexpr (MU == 0) {
    const int base = h - (c.x >> 1);
    const int xf = (c.x + 1 == g.L[0]) ? 0 : c.x + 1;
    const int xb = (c.x == 0) ? g.L[0] - 1 : c.x - 1;
    hf = base + (xf >> 1);
    hb = base + (xb >> 1);
  } else if constexpr (MU == 1) {
    hf = (c.y + 1 == g.L[1]) ? h - (g.L[1] - 1) * g.sy : h + g.sy;
    hb = (c.y == 0) ? h + (g.L[1] - 1) * g.sy : h - g.sy;
  } else if constexpr (MU == 2) {
    hf = (c.z + 1 == g.L[2]) ? h - (g.L[2] - 1) * g.sz : h + g.sz;
    hb = (c.z == 0) ? h + (g.L[2] - 1) * g.sz : h - g.sz;
  } else {
    hf = (c.t + 1 == g.L[3]) ? h - (g.L[3] - 1) * g.st : h + g.st;
    hb = (c.t == 0) ? h + (g.L[3] - 1) * g.st : h - g.st;
  }
  {  // forward: (1 -/+ gamma) U_mu(x) phi(x + mu)
    cx<T> f[4][3], h1[3], h2[3], u[9], w1[3], w2[3];
    load_spinor<MU, FWD_MINUS>(g, in, npar, hf, f);
    project<MU, FWD_MINUS>(f, h1, h2);
    load_link(g, U, MU, par, h, u);
#pragma unroll
    for (int r = 0; r < 3; r++) {
      w1[r] = u[3 * r] * h1[0] + u[3 * r + 1] * h1[1] + u[3 * r + 2] * h1[2];
      w2[r] = u[3 * r] * h2[0] + u[3 * r + 1] * h2[1] + u[3 * r + 2] * h2[2];
    }
    accumulate<MU, FWD_MINUS>(a, w1, w2);
  }
  {  // backward: (1 +/- gamma) U_mu(x - mu)^dag phi(x - mu)
    cx<T> f[4][3], h1[3], h2[3], u[9], w1[3], w2[3];
    load_spinor<MU, !FWD_MINUS>(g, in, npar, hb, f);
    project<MU, !FWD_MINUS>(f, h1, h2);
    load_link(g, U, MU, npar, hb, u);
#pragma unroll
    for (int r = 0; r < 3; r++) {
      w1[r] = cmulc(u[r], h1[0]) + cmulc(u[3 + r], h1[1]) + cmulc(u[6 + r], h1[2]);
      w2[r] = cmulc(u[r], h2[0]) + cmulc(u[3 + r], h2[1]) + cmulc(u[6 + r], h2[2]);
    }
    accumulate<MU, !FWD_MINUS>(a, w1, w2);
  }
}

// out = D in, H in, D^dag in, or b - D in, over the sites of parities
// [par0, par0 + npar), with optional reduction epilogues.
template <typename S, int OP, int EPI>
__global__ __launch_bounds__(256) void k_dslash(Geom g, S* __restrict__ out, const S* __restrict__ in,
                                                const S* __restrict__ U, double kappa, const S* __restrict__ aux,
                                                double* __restrict__ partials, int par0, int nbp,
                                                const int* __restrict__ active, int ftz) {
  using T = typename Traits<S>::T;
  if (active && *active == 0) return;
  const int par = par0 + blockIdx.x / nbp;
  const int h = (blockIdx.x % nbp) * 256 + threadIdx.x;
  constexpr bool DAG = (OP == kOpDdag || OP == kOpHdag);
  constexpr int NV = (EPI == kEpiNone) ? 1 : (EPI == kEpiDotAux ? 2 : (EPI == kEpiTS ? 4 : 1));
  double red[NV];
#pragma unroll
  for (int i = 0; i < NV; i++) red[i] = 0.0;
  if (h < g.Vh) {
    const Coord c = decode(g, par, h);
    cx<T> a[4][3];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int cc = 0; cc < 3; cc++) a[s][cc] = cx<T>(0, 0);
    hop_dir<0, DAG>(g, in, U, par, h, c, a);
    hop_dir<1, DAG>(g, in, U, par, h, c, a);
    hop_dir<2, DAG>(g, in, U, par, h, c, a);
    hop_dir<3, DAG>(g, in, U, par, h, c, a);
    const T k = (T)kappa;
    T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int cc = 0; cc < 3; cc++) {
        const int comp = 3 * s + cc;
        const size_t idx = sp_index(g, par, h, comp);
        cx<T> o, ctr;
        if constexpr (OP == kOpH || OP == kOpHdag) {
          o = a[s][cc];
        } else {
          ctr = Traits<S>::load(in + idx);
          o = ctr - k * a[s][cc];
          if constexpr (EPI == kEpiResid) o = Traits<S>::load(aux + idx) - o;
        }
        const S st = Traits<S>::pack(o, ftz);
        out[idx] = st;
        if constexpr (EPI != kEpiNone) {
          // reductions see the stored value
          const cx<T> os = Traits<S>::load(&st);
          if constexpr (EPI == kEpiDotAux) {  // (aux, out) = sum conj(aux) out
            const cx<T> r = Traits<S>::load(aux + idx);
            acc0 += r.re * os.re + r.im * os.im;
            acc1 += r.re * os.im - r.im * os.re;
          } else if constexpr (EPI == kEpiTS) {  // (t, s) with t = out, s = in; |t|^2, |s|^2
            acc0 += os.re * ctr.re + os.im * ctr.im;
            acc1 += os.re * ctr.im - os.im * ctr.re;
            acc2 += norm2(os);
            acc3 += norm2(ctr);
          } else {
            acc0 += norm2(os);
          }
        }
      }
    if constexpr (EPI == kEpiDotAux) { red[0] = acc0; red[1] = acc1; }
    if constexpr (EPI == kEpiTS) { red[0] = acc0; red[1] = acc1; red[2] = acc2; red[3] = acc3; }
    if constexpr (EPI == kEpiResid) { red[0] = acc0; }
  }
  if constexpr (EPI != kEpiNone) block_reduce_store<NV>(red, partials, blockIdx.x);
}

template <typename S>
static void launch_dslash_t(const Geom& g, int op, int epi, void* out, const void* in, const void* U, double kappa,
                            const void* aux, double* partials, int par0, int npar, const int* active, int ftz,
                            hipStream_t st) {
  const int nbp = (g.Vh + 255) / 256;
  dim3 grid(nbp * npar), block(256);
  S* o = (S*)out;
  const S* i = (const S*)in;
  const S* u = (const S*)U;
  const S* x = (const S*)aux;
#define QCD_LAUNCH(OPV, EPIV) \
  hipLaunchKernelGGL((k_dslash<S, OPV, EPIV>), grid, block, 0, st, g, o, i, u, kappa, x, partials, par0, nbp, active, ftz)
  if (epi == kEpiNone) {
    switch (op) {
      case kOpD: QCD_LAUNCH(kOpD, kEpiNone); break;
      case kOpH: QCD_LAUNCH(kOpH, kEpiNone); break;
      case kOpDdag: QCD_LAUNCH(kOpDdag, kEpiNone); break;
      default: QCD_LAUNCH(kOpHdag, kEpiNone); break;
    }
  } else if (epi == kEpiDotAux) {
    QCD_LAUNCH(kOpD, kEpiDotAux);
  } else if (epi == kEpiTS) {
    QCD_LAUNCH(kOpD, kEpiTS);
  } else {
    QCD_LAUNCH(kOpD, kEpiResid);
  }
#undef QCD_LAUNCH
}

void launch_dslash(int prec, const Geom& g, int op, int epi, void* out, const void* in, const void* U, double kappa,
                   const void* aux, double* partials, int par0, int npar, const int* active, int ftz,
                   hipStream_t st) {
  if (prec == kFP64)
    launch_dslash_t<double2>(g, op, epi, out, in, U, kappa, aux, partials, par0, npar, active, ftz, st);
  else if (prec == kFP32)
    launch_dslash_t<float2>(g, op, epi, out, in, U, kappa, aux, partials, par0, npar, active, ftz, st);
  else
    launch_dslash_t<__half2>(g, op, epi, out, in, U, kappa, aux, partials, par0, npar, active, ftz, st);
}

int dslash_partial_rows(const Geom& g, int npar) { return ((g.Vh + 255) / 256) * npar; }

}  // namespace qcd
