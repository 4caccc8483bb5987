// Gauge-covariant parallel-transport network (learned right preconditioner).
//
// A layer maps C_in spinor fields to C_out fields,
//   out_j(x) = sum_i sum_p W[p][j][i] (T_p psi_i)(x),
// over nine paths p = 0, +x, -x, +y, -y, +z, -z, +t, -t with
//   (T_{+mu} psi)(x) = U_mu(x) psi(x + mu),  (T_{-mu} psi)(x) = U_mu(x - mu)^dag psi(x - mu),
// and W[p][j][i] a complex 4x4 spin matrix; the network composes its layers
// linearly, so it is gauge covariant and a fixed linear operator.
//
// GPU form.  For every (site, colour) column n the transported inputs are
// written once as a real vector X[n][k], k = (re/im, p, i, spin), in BF16.
// The channel mixing is then the real GEMM
//   [out_re; out_im](16 x N) = A (16 x Kp) X^T,  A = [[Wr, -Wi], [Wi, Wr]],
// run on MFMA 16x16x16 BF16 tiles with FP32 accumulation (rows padded to 16,
// Kp = 2K rounded up to 16).  The backward pass uses A^T for dX (MFMA), the
// adjoint transports (T_{+mu}^dag = T_{-mu} for unitary links) as a gather,
// and an MFMA reduction over columns for dW = dOut X^H.  Activations are
// native FP32 spinor fields; links are the handle's native FP32 copy.  The
// fused inference layer forms X in registers instead and multiplies on the
// 16x16x32 BF16 instruction (K padded to 32).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "qcd.h"
#include "internal.h"
#include "half_ops.h"

namespace qcd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));    // BF16 bits, 8 k of one lane
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));  // the 16x16x32 BF16 operand type
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (the hardware's conversion).
__device__ __forceinline__ short to_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }
__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// Element type E of the two-pass GEMM operands (X, A, DO): BF16 (as short
// bits) on the 16x16x16 BF16 matrix-core instruction, or FP32 on the 16x16x4
// FP32 one (the network's FP32 mixing mode).  In both a lane supplies four
// consecutive k of its row or column: one BF16 instruction takes all four,
// or four FP32 instructions take one each (the sum over k is the same).
template <typename E> struct Mix;
template <> struct Mix<short> {
  using V4 = bf16x4;
  static __device__ __forceinline__ short cvt(float f) { return to_bf16(f); }
  static __device__ __forceinline__ f32x4 mma(V4 a, V4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
template <> struct Mix<float> {
  using V4 = f32x4;
  static __device__ __forceinline__ float cvt(float f) { return f; }
  static __device__ __forceinline__ f32x4 mma(V4 a, V4 b, f32x4 c) {
#pragma unroll
    for (int q = 0; q < 4; q++) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[q], c, 0, 0, 0);
    return c;
  }
};

struct PtcLayerDev {
  int cin, cout, K, M, Kp;  // K = 9*cin*4 complex inputs, M = cout*4 complex outputs, Kp = 2K rounded to 16
};

// neighbour half index of (par, h) one step along +mu (dir > 0) or -mu
__device__ __forceinline__ int nbr(const Geom& g, int h, const Coord& c, int mu, int dir) {
  if (mu == 0) {
    const int base = h - (c.x >> 1);
    const int xn = dir > 0 ? ((c.x + 1 == g.L[0]) ? 0 : c.x + 1) : ((c.x == 0) ? g.L[0] - 1 : c.x - 1);
    return base + (xn >> 1);
  }
  const int cm = mu == 1 ? c.y : (mu == 2 ? c.z : c.t);
  const int st = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
  if (dir > 0) return (cm + 1 == g.L[mu]) ? h - (g.L[mu] - 1) * st : h + st;
  return (cm == 0) ? h + (g.L[mu] - 1) * st : h - st;
}

// out = U f (dag = 0) or U^dag f (dag = 1), colour index of f[s][c]
__device__ __forceinline__ void su3_apply(const cx<float> (&u)[9], const cx<float> (&f)[12], bool dag,
                                          cx<float> (&o)[12]) {
#pragma unroll
  for (int s = 0; s < 4; s++)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      cx<float> acc(0, 0);
#pragma unroll
      for (int b = 0; b < 3; b++) acc = acc + (dag ? cmulc(u[3 * b + a], f[3 * s + b]) : u[3 * a + b] * f[3 * s + b]);
      o[3 * s + a] = acc;
    }
}

__device__ __forceinline__ size_t col_of(const Geom& g, int par, int h) { return ((size_t)par * g.nb * 64 + h) * 3; }
__device__ __forceinline__ size_t ncols(const Geom& g) { return (size_t)2 * g.nb * 64 * 3; }
// Element (column n, k) of a column-major operand of the two-pass form (X in
// BF16, DX in FP32), stored k-tile-major: per batch and k-tile the 16 k-values
// of each column are contiguous, so the 16 columns x 16 k of one matrix-core
// tile are one contiguous segment.  nc = columns per batch entry, nk = Kp / 16.
__device__ __forceinline__ size_t xidx(size_t nc, int nk, size_t n, int k) {
  const size_t b = n / nc, col = n - b * nc;
  return ((b * nk + (k >> 4)) * nc + col) * 16 + (k & 15);
}

// ---------------------------------------------------------------------------
// Forward transport: X (BF16 or FP32) at (n, k), n = b * ncols + column (site, colour),
// k = reim*K + (p*cin + i)*4 + spin; k in [2K, Kp) and padding sites are zero.
template <typename E>
__global__ __launch_bounds__(256) void k_ptc_transport(Geom g, PtcLayerDev L, const float2* __restrict__ act,
                                                       const float2* __restrict__ U, int recon, E* __restrict__ X) {
  const int b = blockIdx.y;
  const int i_site = blockIdx.x * 256 + threadIdx.x;  // over 2 * nb * 64 (padding included)
  const int per = g.nb * 64;
  if (i_site >= 2 * per) return;
  const int par = i_site >= per, h = i_site - par * per;
  const size_t nc = ncols(g);
  const int nk = L.Kp / 16;
  const size_t n0 = (size_t)b * nc + col_of(g, par, h);  // column of colour 0
  if (h >= g.Vh) {  // padding site: zero columns
    for (int c = 0; c < 3; c++)
      for (int k = 0; k < L.Kp; k++) X[xidx(nc, nk, n0 + c, k)] = 0;
    return;
  }
  const Coord c = decode(g, par, h);
  const size_t fstride = spinor_elems(g);
  for (int k = 2 * L.K; k < L.Kp; k++)
    for (int cc = 0; cc < 3; cc++) X[xidx(nc, nk, n0 + cc, k)] = 0;
  for (int i = 0; i < L.cin; i++) {
    const float2* f = act + ((size_t)b * L.cin + i) * fstride;
    for (int p = 0; p < 9; p++) {
      cx<float> in[12], t[12];
      if (p == 0) {
        load_site(f, g, par, h, t);
      } else {
        const int mu = (p - 1) >> 1;
        const bool fwd = ((p - 1) & 1) == 0;
        const int hn = nbr(g, h, c, mu, fwd ? 1 : -1);
        load_site(f, g, par ^ 1, hn, in);
        cx<float> u[9];
        if (fwd) load_link_any(g, U, recon, mu, par, h, u);       // U_mu(x)
        else load_link_any(g, U, recon, mu, par ^ 1, hn, u);      // U_mu(x - mu)^dag
        su3_apply(u, in, !fwd, t);
      }
      const int k0 = (p * L.cin + i) * 4;
      for (int cc = 0; cc < 3; cc++) {
        typename Mix<E>::V4 re, im;
#pragma unroll
        for (int s = 0; s < 4; s++) {
          re[s] = Mix<E>::cvt(t[3 * s + cc].re);
          im[s] = Mix<E>::cvt(t[3 * s + cc].im);
        }
        // k0 and K are multiples of 4, so each group of 4 stays in one k-tile
        *reinterpret_cast<typename Mix<E>::V4*>(X + xidx(nc, nk, n0 + cc, k0)) = re;
        *reinterpret_cast<typename Mix<E>::V4*>(X + xidx(nc, nk, n0 + cc, L.K + k0)) = im;
      }
    }
  }
}

// A[16][Kp] (BF16 or FP32) from the complex weights W[p][j][i][s'][s] of one layer.
template <typename E>
__global__ void k_ptc_prep_A(PtcLayerDev L, const float2* __restrict__ W, E* __restrict__ A) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 16 * L.Kp) return;
  const int r = idx / L.Kp, k = idx % L.Kp;
  float v = 0.0f;
  const bool rre = r < L.M, rim = r >= L.M && r < 2 * L.M;
  const bool kre = k < L.K, kim = k >= L.K && k < 2 * L.K;
  if ((rre || rim) && (kre || kim)) {
    const int row = rre ? r : r - L.M;       // (j, s')
    const int kk = kre ? k : k - L.K;         // (p, i, s)
    const int j = row >> 2, sp = row & 3;
    const int p = kk / (L.cin * 4), i = (kk / 4) % L.cin, s = kk & 3;
    const float2 w = W[(((size_t)(p * L.cout + j) * L.cin + i) * 4 + sp) * 4 + s];
    if (rre && kre) v = w.x;
    else if (rre && kim) v = -w.y;
    else if (rim && kre) v = w.y;
    else v = w.x;
  }
  A[idx] = Mix<E>::cvt(v);
}

// Channel mixing: out[b][j] (native FP32 fields) = layer(X).  One wave per
// tile of 16 columns; A fragments stay in registers.
template <typename E>
__global__ __launch_bounds__(256) void k_ptc_mix(Geom g, PtcLayerDev L, const E* __restrict__ X,
                                                 const E* __restrict__ A, float2* __restrict__ out, int nbatch) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nwaves = gridDim.x * 4;
  const size_t N = ncols(g);
  const size_t ntiles = (N * nbatch) / 16;  // N is a multiple of 192
  const int nk = L.Kp / 16;
  typename Mix<E>::V4 af[9];
#pragma unroll
  for (int kt = 0; kt < 9; kt++)
#pragma unroll
    for (int q = 0; q < 4; q++) af[kt][q] = kt < nk ? A[(lane % 16) * L.Kp + kt * 16 + 4 * (lane / 16) + q] : 0;
  const size_t fstride = spinor_elems(g);
  for (size_t tile = wave; tile < ntiles; tile += nwaves) {
    const size_t n = tile * 16 + (lane % 16);
    f32x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kt = 0; kt < 9; kt++) {
      if (kt >= nk) break;
      const typename Mix<E>::V4 bf =
          *reinterpret_cast<const typename Mix<E>::V4*>(X + xidx(N, nk, n, kt * 16 + 4 * (lane / 16)));
      acc = Mix<E>::mma(af[kt], bf, acc);
    }
    // lane holds rows 4*(lane/16) + q of column n
    const int b = (int)(n / N);
    const size_t nn = n - (size_t)b * N;
    const int site = (int)(nn / 3), cc = (int)(nn % 3);
    const int per = g.nb * 64;
    const int par = site >= per, h = site - par * per;
    if (h >= g.Vh) continue;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int r = 4 * (lane / 16) + q;
      if (r >= 2 * L.M) continue;
      const int row = r < L.M ? r : r - L.M;
      const int j = row >> 2, sp = row & 3;
      float* dst = reinterpret_cast<float*>(out + ((size_t)b * L.cout + j) * fstride + sp_block(g, par, h) +
                                            sp_off<float2>(3 * sp + cc, h & 63));
      dst[r < L.M ? 0 : 1] = acc[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Fused forward layer (inference): the transported inputs are formed in
// registers and fed to the matrix cores directly, so nothing but the
// activations and links crosses HBM.
//
// Column ordering: a wave takes 16 sites (one per lane % 16) and all three
// colours (three accumulators).  The products run on the 16 x 16 x 32 BF16
// instruction; K is ordered by position q of a (path, input channel) pair,
// 8 k each: k = 8 q + 4 sh + 2 s_lo + re/im for spin s = 2 sh + s_lo.
// Position q holds channel i = q % C_in of path p = (q / C_in + 1) mod 9, so
// the hops come first, the forward and backward hop of one direction side
// by side, and the identity path last.  K-tile kt holds positions 4 kt + G,
// lane group G = lane / 16 supplying all 8 k of its pair: a lane transports
// a whole spinor, loading and rebuilding the link once for both spin halves;
// with C_in = 2 the direction of a k-tile is the same for the whole wave, and
// the last k-tile is the identity path only.  Output rows are
// r = (j * 2 + sh') * 4 + s'_lo * 2 + re/im, so lane group G ends up holding
// channel j = G / 2, spins 2 (G % 2) and 2 (G % 2) + 1 of its site for all
// three colours.

// K of the fused layer's weight operand: 2K rounded up to whole 32-wide k-tiles.
__host__ __device__ inline int fused_kp(const PtcLayerDev& L) { return ((2 * L.K + 31) / 32) * 32; }
// path of pair position q
__host__ __device__ inline int fused_path(int q, int cin) { return (q / cin + 1) % 9; }

// A for the fused ordering, from W[p][j][i][s'][s] of one layer (rows of fused_kp(L)).
__global__ void k_ptc_prep_Af(PtcLayerDev L, const float2* __restrict__ W, short* __restrict__ A) {
  const int kf = fused_kp(L);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 16 * kf) return;
  const int r = idx / kf, k = idx % kf;
  const int j = r >> 3, spo = ((r >> 2) & 1) * 2 + ((r >> 1) & 1), ro = r & 1;
  const int q = k >> 3, e = k & 7;
  float v = 0.0f;
  if (j < L.cout && q < 9 * L.cin) {
    const int p = fused_path(q, L.cin), i = q % L.cin, s = (e >> 2) * 2 + ((e >> 1) & 1), ri = e & 1;
    const float2 w = W[(((size_t)(p * L.cout + j) * L.cin + i) * 4 + spo) * 4 + s];
    v = ro == ri ? w.x : (ro == 0 ? -w.y : w.y);
  }
  A[idx] = to_bf16(v);
}

// The transported spinor of one (path, input channel) pair in binary16 form
// (FP16 activations and links): the neighbour's three 16-byte granules, the
// link's row 2 rebuilt in binary16, and U v / U^dag v as exact binary16
// products summed in FP32 (the Wilson operator's FP16 arithmetic).  The lanes
// of a wave take different paths (forward and backward hops), so each lane
// selects its entries and signs into the one forward product form.
template <int CIN>
__device__ __forceinline__ void fused_transport_h(const Geom& g, const __half2* __restrict__ in,
                                                  const __half2* __restrict__ U, int recon, int b, int p, int i,
                                                  int par, int h, const Coord& c, size_t fstride,
                                                  cx<float> (&t)[4][3]) {
  using Gr = typename Lay<__half2>::Gran;  // 4 complex components
  const __half2* f = in + ((size_t)b * CIN + i) * fstride;
  const int mu = (p - 1) >> 1;  // p = 1..8
  const bool fwd = ((p - 1) & 1) == 0;
  const int sh_idx = nbr(g, h, c, mu, fwd ? 1 : -1);
  const __half2* fb = f + sp_block(g, par ^ 1, sh_idx) + (sh_idx & 63) * 4;
  h2v v[4][3];  // v[spin][colour]: component 3 spin + colour
#pragma unroll
  for (int j = 0; j < 3; j++) {
    const Gr q = *reinterpret_cast<const Gr*>(fb + j * 64 * 4);
#pragma unroll
    for (int e = 0; e < 4; e++) v[(4 * j + e) / 3][(4 * j + e) % 3] = h2_of(q.s[e]);
  }
  // U_mu(x) (forward) or U_mu(x - mu) (backward, applied as its adjoint)
  const int lp = fwd ? par : par ^ 1, lh = fwd ? h : sh_idx, lane = lh & 63;
  h2v u[9];
  if (recon) {
    const __half2* lb = U + lk_block<6>(g, mu, lp, lh);
    const Gr q = *reinterpret_cast<const Gr*>(lb + lane * 4);
    const __half2* tl = lb + 4 * 64 + lane * 2;
#pragma unroll
    for (int k = 0; k < 4; k++) u[k] = h2_of(q.s[k]);
    u[4] = h2_of(tl[0]);
    u[5] = h2_of(tl[1]);
    h_third_row(u);
  } else {
    const __half2* lb = U + lk_block<9>(g, mu, lp, lh);
    const Gr q0 = *reinterpret_cast<const Gr*>(lb + lane * 4);
    const Gr q1 = *reinterpret_cast<const Gr*>(lb + 64 * 4 + lane * 4);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      u[k] = h2_of(q0.s[k]);
      u[4 + k] = h2_of(q1.s[k]);
    }
    u[8] = h2_of(lb[8 * 64 + lane]);
  }
  // Entry (r, b) of U, or of U^dag read as conj(u[3b + r]), with the sign
  // flips of each form applied per lane: the same products in the same order
  // as h_mult, without running both forms.
  const uint32_t pm = fwd ? 0x80000000u : 0u;  // (re, -im) forward, (re, im) backward
  const uint32_t qm = fwd ? 0u : 0x8000u;      // (im, re) forward, (-im, re) backward
  HLink<false> L;
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int bb = 0; bb < 3; bb++) {
      // both entries as values first: a conditional of two array elements
      // would select an address and index the array at run time
      const uint32_t ef = __builtin_bit_cast(uint32_t, u[3 * r + bb]);
      const uint32_t eb = __builtin_bit_cast(uint32_t, u[3 * bb + r]);
      const uint32_t a = fwd ? ef : eb;
      L.p[3 * r + bb] = __builtin_bit_cast(h2v, a ^ pm);
      L.q[3 * r + bb] = __builtin_bit_cast(h2v, ((a >> 16) | (a << 16)) ^ qm);
    }
#pragma unroll
  for (int s_ = 0; s_ < 4; s_++) h_mult<false>(L, v[s_], t[s_]);
}

// out[b][j] = oscale * sum_{p,i} W[p][j][i] T_p in[b][i] for batch b = blockIdx.y;
// grid.x = 2 * nb (one 64-site block of one parity per workgroup).  Batches
// whose solver has stopped (scal[b].active == 0) are skipped when scal is given.
template <typename SA, typename SL, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_ptc_fused(Geom g, const SA* __restrict__ in, SA* __restrict__ out,
                                                   const SL* __restrict__ U, int recon, const short* __restrict__ A,
                                                   int Kf, float oscale, const Scalars* __restrict__ scal, int ftz) {
  constexpr int NK = (9 * CIN + 3) / 4;  // 32-wide k-tiles: four (path, channel) pairs each
  const int b = blockIdx.y;
  if (scal && !scal[b].active) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = lane >> 4, n = lane & 15;
  const int par = blockIdx.x >= g.nb, hb = blockIdx.x - par * g.nb;
  const int h_raw = hb * 64 + w * 16 + n;
  const bool valid = h_raw < g.Vh;
  const int h = valid ? h_raw : 0;  // padding lanes compute on site 0 and store nothing
  const Coord c = decode(g, par, h);
  const size_t fstride = spinor_elems(g);
  bf16x8 af[NK];
#pragma unroll
  for (int kt = 0; kt < NK; kt++) {
    const s16x8 a8 = *reinterpret_cast<const s16x8*>(A + (lane & 15) * Kf + kt * 32 + 8 * G);
    af[kt] = __builtin_bit_cast(bf16x8, a8);
  }
  f32x4 acc[3];
#pragma unroll
  for (int cc = 0; cc < 3; cc++) acc[cc] = (f32x4){0, 0, 0, 0};
#pragma unroll
  for (int kt = 0; kt < NK; kt++) {
    const int q = 4 * kt + G;  // pair position: channel q % C_in of path fused_path(q, C_in)
    cx<float> t[4][3];         // transported spins 0..3, colours 0..2
#pragma unroll
    for (int s_ = 0; s_ < 4; s_++)
#pragma unroll
      for (int cc = 0; cc < 3; cc++) t[s_][cc] = cx<float>(0, 0);
    if (kt == NK - 1) {  // the identity path (positions past 9 C_in are padding)
      if (q < 9 * CIN) {
        const SA* fb = in + ((size_t)b * CIN + q % CIN) * fstride + sp_block(g, par, h);
#pragma unroll
        for (int s_ = 0; s_ < 4; s_++)
#pragma unroll
          for (int cc = 0; cc < 3; cc++) t[s_][cc] = Traits<SA>::load(fb + sp_off<SA>(3 * s_ + cc, h & 63));
      }
    } else if constexpr (std::is_same<SA, __half2>::value && std::is_same<SL, __half2>::value) {
      fused_transport_h<CIN>(g, in, U, recon, b, q / CIN + 1, q % CIN, par, h, c, fstride, t);
    } else {
      const int p = q / CIN + 1, i = q % CIN;  // a hop, p = 1..8
      const SA* f = in + ((size_t)b * CIN + i) * fstride;
      const int mu = (p - 1) >> 1;
      const bool fwd = ((p - 1) & 1) == 0;
      const int hn = nbr(g, h, c, mu, fwd ? 1 : -1);
      const SA* fb = f + sp_block(g, par ^ 1, hn);
      cx<float> v[4][3], u[9];
#pragma unroll
      for (int s_ = 0; s_ < 4; s_++)
#pragma unroll
        for (int cc = 0; cc < 3; cc++) v[s_][cc] = Traits<SA>::load(fb + sp_off<SA>(3 * s_ + cc, hn & 63));
      const int lp = fwd ? par : par ^ 1, lh = fwd ? h : hn;  // U_mu(x) or U_mu(x - mu)
      load_link_any(g, U, recon, mu, lp, lh, u);
#pragma unroll
      for (int s_ = 0; s_ < 4; s_++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
          cx<float> acc_(0, 0);
#pragma unroll
          for (int bb = 0; bb < 3; bb++)
            acc_ = acc_ + (fwd ? u[3 * a + bb] * v[s_][bb] : cmulc(u[3 * bb + a], v[s_][bb]));
          t[s_][a] = acc_;
        }
    }
#pragma unroll
    for (int cc = 0; cc < 3; cc++) {
      // k = 8 q + 4 sh + 2 s_lo + re/im; the hardware's round-to-nearest-even
      // conversion, two values per instruction
      u32x4 bw;
#pragma unroll
      for (int s_ = 0; s_ < 4; s_++) {
        const f32x2 f = {valid ? t[s_][cc].re : 0.0f, valid ? t[s_][cc].im : 0.0f};
        bw[s_] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
      }
      acc[cc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kt], __builtin_bit_cast(bf16x8, bw), acc[cc], 0, 0, 0);
    }
  }
  const int j = G >> 1, sh = G & 1;
  if (!valid || j >= COUT) return;
  SA* ob = out + ((size_t)b * COUT + j) * fstride + sp_block(g, par, h);
#pragma unroll
  for (int sl = 0; sl < 2; sl++)
#pragma unroll
    for (int cc = 0; cc < 3; cc++) {
      const cx<float> o(oscale * acc[cc][2 * sl], oscale * acc[cc][2 * sl + 1]);
      ob[sp_off<SA>(3 * (2 * sh + sl) + cc, h & 63)] = Traits<SA>::pack(o, ftz);
    }
}

// ---------------------------------------------------------------------------
// Backward.

// dOut (native FP32 fields) -> DO[b][n][16] in E, real form (re rows, im rows, zeros).
template <typename E>
__global__ __launch_bounds__(256) void k_ptc_dout_mix(Geom g, PtcLayerDev L, const float2* __restrict__ dout,
                                                      E* __restrict__ DO) {
  const int b = blockIdx.y;
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  const int per = g.nb * 64;
  if (i_site >= 2 * per) return;
  const int par = i_site >= per, h = i_site - par * per;
  E* d = DO + ((size_t)b * ncols(g) + col_of(g, par, h)) * 16;
  const size_t fstride = spinor_elems(g);
  for (int cc = 0; cc < 3; cc++) {
    E row[16];
#pragma unroll
    for (int r = 0; r < 16; r++) row[r] = 0;
    if (h < g.Vh) {
      for (int j = 0; j < L.cout; j++) {
        cx<float> f[12];
        load_site(dout + ((size_t)b * L.cout + j) * fstride, g, par, h, f);
        for (int sp = 0; sp < 4; sp++) {
          row[4 * j + sp] = Mix<E>::cvt(f[3 * sp + cc].re);
          row[L.M + 4 * j + sp] = Mix<E>::cvt(f[3 * sp + cc].im);
        }
      }
    }
    for (int r = 0; r < 16; r += 4) {
      typename Mix<E>::V4 v = {row[r], row[r + 1], row[r + 2], row[r + 3]};
      *reinterpret_cast<typename Mix<E>::V4*>(d + (size_t)cc * 16 + r) = v;
    }
  }
}

// DX[b][n][k] (FP32) = sum_r A[r][k] DO[b][n][r]: one MFMA per (k tile, column tile).
template <typename E>
__global__ __launch_bounds__(256) void k_ptc_mix_dx(Geom g, PtcLayerDev L, const E* __restrict__ DO,
                                                    const E* __restrict__ A, float* __restrict__ DX, int nbatch) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nwaves = gridDim.x * 4;
  const size_t N = ncols(g) * nbatch;
  const size_t ntiles = N / 16;
  const int nk = L.Kp / 16;
  for (size_t tile = wave; tile < ntiles; tile += nwaves) {
    const size_t n = tile * 16 + (lane % 16);
    const size_t nc = ncols(g);
    const typename Mix<E>::V4 bf = *reinterpret_cast<const typename Mix<E>::V4*>(DO + n * 16 + 4 * (lane / 16));
    for (int kt = 0; kt < nk; kt++) {
      typename Mix<E>::V4 at;  // A^T tile: row = k, column = r
#pragma unroll
      for (int q = 0; q < 4; q++) at[q] = A[(4 * (lane / 16) + q) * L.Kp + kt * 16 + (lane % 16)];
      f32x4 acc = {0, 0, 0, 0};
      acc = Mix<E>::mma(at, bf, acc);
      // lane holds rows k = kt*16 + 4*(lane/16) + q of column n
      *reinterpret_cast<f32x4*>(DX + xidx(nc, nk, n, kt * 16 + 4 * (lane / 16))) = acc;
    }
  }
}

// dIn_i(y) = sum_p (T_p^dag dX_{p,i})(y): p = 0 identity; +mu: U_mu(y-mu)^dag dX(y-mu); -mu: U_mu(y) dX(y+mu).
__global__ __launch_bounds__(256) void k_ptc_transport_adj(Geom g, PtcLayerDev L, const float* __restrict__ DX,
                                                           const float2* __restrict__ U, int recon,
                                                           float2* __restrict__ din) {
  const int b = blockIdx.y;
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  if (i_site >= 2 * g.Vh) return;
  const int par = i_site >= g.Vh, h = i_site - par * g.Vh;
  const Coord c = decode(g, par, h);
  const size_t fstride = spinor_elems(g);
  const size_t nc = ncols(g);
  const int nk = L.Kp / 16;
  for (int i = 0; i < L.cin; i++) {
    cx<float> acc[12];
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = cx<float>(0, 0);
    for (int p = 0; p < 9; p++) {
      int sp = par, sh = h;  // site whose dX column is read
      bool dag = false;
      int mu = -1;
      if (p > 0) {
        mu = (p - 1) >> 1;
        const bool fwd = ((p - 1) & 1) == 0;
        sp = par ^ 1;
        sh = nbr(g, h, c, mu, fwd ? -1 : 1);  // +mu path reads y - mu, -mu path reads y + mu
        dag = fwd;
      }
      cx<float> f[12];
      const int k0 = (p * L.cin + i) * 4;
      const size_t n0 = (size_t)b * nc + col_of(g, sp, sh);
#pragma unroll
      for (int cc = 0; cc < 3; cc++) {
        const f32x4 re = *reinterpret_cast<const f32x4*>(DX + xidx(nc, nk, n0 + cc, k0));
        const f32x4 im = *reinterpret_cast<const f32x4*>(DX + xidx(nc, nk, n0 + cc, L.K + k0));
#pragma unroll
        for (int s = 0; s < 4; s++) f[3 * s + cc] = cx<float>(re[s], im[s]);
      }
      if (p == 0) {
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = acc[k] + f[k];
      } else {
        cx<float> u[9], t[12];
        if (dag) load_link_any(g, U, recon, mu, sp, sh, u);   // U_mu(y - mu)^dag
        else load_link_any(g, U, recon, mu, par, h, u);       // U_mu(y)
        su3_apply(u, f, dag, t);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = acc[k] + t[k];
      }
    }
    float2* dst = din + ((size_t)b * L.cin + i) * fstride;
    float2* bb = dst + sp_block(g, par, h);
#pragma unroll
    for (int k = 0; k < 12; k++) bb[sp_off<float2>(k, h & 63)] = make_float2(acc[k].re, acc[k].im);
  }
}

// G partials: Gp[wave][16][Kp] = sum over the wave's columns of DO[n][r] X[n][k].
template <typename E>
__global__ __launch_bounds__(256) void k_ptc_mix_dw(Geom g, PtcLayerDev L, const E* __restrict__ DO,
                                                    const E* __restrict__ X, float* __restrict__ Gp, int nbatch) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nwaves = gridDim.x * 4;
  const size_t N = ncols(g) * nbatch;
  const size_t ntiles = N / 16;
  const int nk = L.Kp / 16;
  const size_t nc = ncols(g);
  f32x4 acc[9];
#pragma unroll
  for (int kt = 0; kt < 9; kt++) acc[kt] = (f32x4){0, 0, 0, 0};
  for (size_t tile = wave; tile < ntiles; tile += nwaves) {
    const size_t n0 = tile * 16;
    typename Mix<E>::V4 a;  // A[r][nn] = DO[n0 + nn][r]: row r = lane % 16, nn = 4*(lane/16) + q
#pragma unroll
    for (int q = 0; q < 4; q++) a[q] = DO[(n0 + 4 * (lane / 16) + q) * 16 + (lane % 16)];
#pragma unroll
    for (int kt = 0; kt < 9; kt++) {
      if (kt >= nk) break;
      typename Mix<E>::V4 bb;  // B[nn][k] = X(n0 + nn, kt*16 + lane % 16)
#pragma unroll
      for (int q = 0; q < 4; q++) bb[q] = X[xidx(nc, nk, n0 + 4 * (lane / 16) + q, kt * 16 + (lane % 16))];
      acc[kt] = Mix<E>::mma(a, bb, acc[kt]);
    }
  }
  // lane holds G[4*(lane/16) + q][kt*16 + lane % 16]
  float* dst = Gp + (size_t)wave * 16 * L.Kp;
#pragma unroll
  for (int kt = 0; kt < 9; kt++) {
    if (kt >= nk) break;
#pragma unroll
    for (int q = 0; q < 4; q++) dst[(size_t)(4 * (lane / 16) + q) * L.Kp + kt * 16 + (lane % 16)] = acc[kt][q];
  }
}

// Sum the wave partials in two fixed-order passes: slice sl adds waves
// sl, sl + kDwSlices, ... for every weight (one thread per weight and slice),
// then the slices are added in order and the complex gradient
// dW = (G00 + G11) + i (G10 - G01) is accumulated into grad in the layout of W.
constexpr int kDwSlices = 64;
__global__ __launch_bounds__(64) void k_ptc_dw_slices(PtcLayerDev L, const float* __restrict__ Gp, int nwaves,
                                                      double* __restrict__ part) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // over M*K complex weights
  if (idx >= L.M * L.K) return;
  const int row = idx / L.K, kk = idx % L.K;
  double g00 = 0, g01 = 0, g10 = 0, g11 = 0;
  for (int w = blockIdx.y; w < nwaves; w += kDwSlices) {
    const float* G = Gp + (size_t)w * 16 * L.Kp;
    g00 += G[(size_t)row * L.Kp + kk];
    g01 += G[(size_t)row * L.Kp + L.K + kk];
    g10 += G[(size_t)(L.M + row) * L.Kp + kk];
    g11 += G[(size_t)(L.M + row) * L.Kp + L.K + kk];
  }
  double* o = part + ((size_t)blockIdx.y * L.M * L.K + idx) * 4;
  o[0] = g00;
  o[1] = g01;
  o[2] = g10;
  o[3] = g11;
}
__global__ void k_ptc_dw_finish(PtcLayerDev L, const double* __restrict__ part, float2* __restrict__ grad) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= L.M * L.K) return;
  const int row = idx / L.K, kk = idx % L.K;
  double g00 = 0, g01 = 0, g10 = 0, g11 = 0;
  for (int sl = 0; sl < kDwSlices; sl++) {
    const double* q = part + ((size_t)sl * L.M * L.K + idx) * 4;
    g00 += q[0];
    g01 += q[1];
    g10 += q[2];
    g11 += q[3];
  }
  const int j = row >> 2, sp = row & 3;
  const int p = kk / (L.cin * 4), i = (kk / 4) % L.cin, s = kk & 3;
  float2& d = grad[(((size_t)(p * L.cout + j) * L.cin + i) * 4 + sp) * 4 + s];
  d.x += (float)(g00 + g11);
  d.y += (float)(g10 - g01);
}

// ---------------------------------------------------------------------------
// Loss |M(r_b) - e_b|^2 / |e_b|^2 (mean over the batch) and its output gradient.

__global__ __launch_bounds__(256) void k_ptc_loss_parts(Geom g, const float2* __restrict__ out,
                                                        const float2* __restrict__ e, double* __restrict__ partials) {
  const int b = blockIdx.y;
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  double red[2] = {0, 0};
  if (i_site < 2 * g.Vh) {
    const int par = i_site >= g.Vh, h = i_site - par * g.Vh;
    const size_t fo = (size_t)b * spinor_elems(g);
    cx<float> o[12], t[12];
    load_site(out + fo, g, par, h, o);
    load_site(e + fo, g, par, h, t);
    float a = 0, n = 0;
    for (int k = 0; k < 12; k++) {
      a += norm2(o[k] - t[k]);
      n += norm2(t[k]);
    }
    red[0] = a;
    red[1] = n;
  }
  block_reduce_store<2>(red, partials + (size_t)b * gridDim.x * 2, blockIdx.x);
}

__global__ void k_ptc_loss_finish(const double* __restrict__ partials, int nrows, int nbatch, double* __restrict__ sums) {
  // sums[b] = (|out-e|^2, |e|^2) for sample blockIdx.x
  double s[2];
  finish_sum<2>(partials + (size_t)blockIdx.x * nrows * 2, nrows, s);
  if (threadIdx.x == 0) {
    sums[2 * blockIdx.x] = s[0];
    sums[2 * blockIdx.x + 1] = s[1];
  }
}

__global__ __launch_bounds__(256) void k_ptc_dout(Geom g, const float2* __restrict__ out, const float2* __restrict__ e,
                                                  const double* __restrict__ sums, int nbatch,
                                                  float2* __restrict__ dout) {
  const int b = blockIdx.y;
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  if (i_site >= 2 * g.Vh) return;
  const int par = i_site >= g.Vh, h = i_site - par * g.Vh;
  const size_t fo = (size_t)b * spinor_elems(g);
  const float c = (float)(2.0 / (nbatch * sums[2 * b + 1]));
  cx<float> o[12], t[12], d[12];
  load_site(out + fo, g, par, h, o);
  load_site(e + fo, g, par, h, t);
  for (int k = 0; k < 12; k++) d[k] = c * (o[k] - t[k]);
  store_site(dout + fo, g, par, h, d, 0);
}

// Per-field |a|^2 and |b|^2 (for the gain |M(v)| / |v| of the network).
__global__ __launch_bounds__(256) void k_ptc_norms(Geom g, const float2* __restrict__ a, const float2* __restrict__ b,
                                                   double* __restrict__ partials) {
  const int bi = blockIdx.y;
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  double red[2] = {0, 0};
  if (i_site < 2 * g.Vh) {
    const int par = i_site >= g.Vh, h = i_site - par * g.Vh;
    const size_t fo = (size_t)bi * spinor_elems(g);
    cx<float> x[12], y[12];
    load_site(a + fo, g, par, h, x);
    load_site(b + fo, g, par, h, y);
    float na = 0, nb = 0;
    for (int k = 0; k < 12; k++) {
      na += norm2(x[k]);
      nb += norm2(y[k]);
    }
    red[0] = na;
    red[1] = nb;
  }
  block_reduce_store<2>(red, partials + (size_t)bi * gridDim.x * 2, blockIdx.x);
}

// Adam on FP32 weights (Kingma & Ba 2015), bias-corrected.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gr = grad[i];
  const float mi = b1 * m[i] + (1 - b1) * gr;
  const float vi = b2 * v[i] + (1 - b2) * gr * gr;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP16 native -> FP32 native and back (for applying the network inside the FP16 solver).
__global__ __launch_bounds__(256) void k_h2f(Geom g, const __half2* __restrict__ src, float2* __restrict__ dst,
                                             float scale) {
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  if (i_site >= 2 * g.Vh) return;
  const int par = i_site >= g.Vh, h = i_site - par * g.Vh;
  const size_t o = (size_t)blockIdx.y * spinor_elems(g);
  cx<float> f[12];
  load_site(src + o, g, par, h, f);
  for (int k = 0; k < 12; k++) f[k] = scale * f[k];
  store_site(dst + o, g, par, h, f, 0);
}
__global__ __launch_bounds__(256) void k_f2h(Geom g, const float2* __restrict__ src, __half2* __restrict__ dst,
                                             int ftz) {
  const int i_site = blockIdx.x * 256 + threadIdx.x;
  if (i_site >= 2 * g.Vh) return;
  const int par = i_site >= g.Vh, h = i_site - par * g.Vh;
  const size_t o = (size_t)blockIdx.y * spinor_elems(g);
  cx<float> f[12];
  load_site(src + o, g, par, h, f);
  store_site(dst + o, g, par, h, f, ftz);
}

}  // namespace qcd

// ===========================================================================
// Host side: the network handle and its C ABI.

using namespace qcd;

struct qcd_ptc {
  const qcd_gauge* gauge;
  Geom g;
  int nlayers;
  int channels[kPtcMaxLayers + 1];
  PtcLayerDev L[kPtcMaxLayers];
  int max_batch;
  size_t nweights;                  // complex weights in total
  size_t woff[kPtcMaxLayers];       // complex offset of each layer's weights
  float2* w;                        // FP32 master weights
  float2* grad;
  float2* adam_m;
  float2* adam_v;
  int adam_step;
  int mix_fp32;                     // 1: the two-pass GEMMs (A, X, DO) in FP32, else BF16
  void* A[kPtcMaxLayers];           // GEMM operands (training ordering), BF16 or FP32
  short* Af[kPtcMaxLayers];         // BF16 GEMM operands (fused inference ordering)
  __half2* act16[kPtcMaxLayers + 1];  // FP16 hidden activations of the solver's applications
  float2* act[kPtcMaxLayers + 1];   // activations (batch x channels native FP32 fields)
  // Buffers of the two-pass form (training, and the FP32 mixing mode), allocated
  // on its first use: a handle that only preconditions never holds them.
  bool two_pass_ready;
  float2* target;                   // training targets (batch fields)
  float2* dact[2];                  // gradient ping-pong buffers
  void* X[kPtcMaxLayers];           // transported inputs per layer (kept for the backward pass), BF16 or FP32
  void* DO;                         // output gradient in the real form, BF16 or FP32
  float* DX;
  float* Gp;
  double* dwp;                      // weight-gradient slices [kDwSlices][M*K][4]
  double* partials;
  double* sums;
  int mix_blocks;
  std::vector<void*> allocs;
};

namespace {

template <typename... A> qcd_status pfail(qcd_status code, const char* fmt, A... a) {
  return (qcd_status)set_error((int)code, fmt, a...);
}
#define PTC_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return pfail(QCD_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));            \
  } while (0)
#define PTC_LAUNCHED()                                                                                  \
  do {                                                                                                  \
    hipError_t e_ = hipGetLastError();                                                                  \
    if (e_ != hipSuccess) return pfail(QCD_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_));        \
  } while (0)

size_t fields_bytes(const Geom& g, size_t nf) { return nf * spinor_elems(g) * sizeof(float2); }
int site_blocks_pad(const Geom& g) { return (2 * g.nb * 64 + 255) / 256; }
int site_blocks(const Geom& g) { return (2 * g.Vh + 255) / 256; }
const float2* links32(const qcd_ptc* n) { return (const float2*)n->gauge->U[kFP32]; }
int recon_of(const qcd_ptc* n, int prec) { return n->gauge->tune[prec].recon; }

qcd_status alloc(qcd_ptc* n, void** p, size_t bytes) {
  PTC_TRY(hipMalloc(p, bytes ? bytes : 256));
  n->allocs.push_back(*p);
  return QCD_OK;
}

void prep_weights(qcd_ptc* n, hipStream_t st) {
  for (int l = 0; l < n->nlayers; l++) {
    const int cnt = 16 * n->L[l].Kp, cntf = 16 * fused_kp(n->L[l]);
    if (n->mix_fp32)
      hipLaunchKernelGGL(k_ptc_prep_A<float>, dim3((cnt + 255) / 256), dim3(256), 0, st, n->L[l],
                         (const float2*)(n->w + n->woff[l]), (float*)n->A[l]);
    else
      hipLaunchKernelGGL(k_ptc_prep_A<short>, dim3((cnt + 255) / 256), dim3(256), 0, st, n->L[l],
                         (const float2*)(n->w + n->woff[l]), (short*)n->A[l]);
    hipLaunchKernelGGL(k_ptc_prep_Af, dim3((cntf + 255) / 256), dim3(256), 0, st, n->L[l],
                       (const float2*)(n->w + n->woff[l]), n->Af[l]);
  }
}

// Widest GEMM operand row of the network, and the rows of a batch element.
int max_kp(const qcd_ptc* n) {
  int m = 16;
  for (int l = 0; l < n->nlayers; l++) m = std::max(m, n->L[l].Kp);
  return m;
}
size_t gemm_rows(const Geom& g) { return (size_t)2 * g.nb * 64 * 3; }

// The two-pass form's buffers (max_batch elements each), on first use.
qcd_status ensure_two_pass(qcd_ptc* n) {
  if (n->two_pass_ready) return QCD_OK;
  const Geom& g = n->g;
  const size_t N = gemm_rows(g), es = n->mix_fp32 ? sizeof(float) : sizeof(short);
  const int maxKp = max_kp(n);
  int maxc = 1;
  for (int l = 0; l <= n->nlayers; l++) maxc = std::max(maxc, n->channels[l]);
  qcd_status rc = QCD_OK;
  // the FP32-mixing inference reuses X[0] for every layer: it takes the widest layer's size
  for (int l = 0; l < n->nlayers && rc == QCD_OK; l++)
    rc = alloc(n, &n->X[l], (size_t)n->max_batch * N * (l == 0 ? maxKp : n->L[l].Kp) * es);
  if (rc == QCD_OK) rc = alloc(n, &n->DO, (size_t)n->max_batch * N * 16 * es);
  if (rc == QCD_OK) rc = alloc(n, (void**)&n->DX, (size_t)n->max_batch * N * maxKp * sizeof(float));
  if (rc == QCD_OK) rc = alloc(n, (void**)&n->target, fields_bytes(g, n->max_batch));
  if (rc == QCD_OK) rc = alloc(n, (void**)&n->dact[0], fields_bytes(g, (size_t)n->max_batch * maxc));
  if (rc == QCD_OK) rc = alloc(n, (void**)&n->dact[1], fields_bytes(g, (size_t)n->max_batch * maxc));
  if (rc) return rc;
  n->two_pass_ready = true;
  return QCD_OK;
}

template <typename SA, typename SL>
void fused_layer(const qcd_ptc* n, int l, int nb, const SA* in, SA* out, const SL* U, float oscale,
                 const Scalars* scal, int ftz, hipStream_t st) {
  const Geom& g = n->g;
  const PtcLayerDev& L = n->L[l];
  const dim3 grid(2 * g.nb, nb), block(256);
  const int recon = recon_of(n, sizeof(SL) == sizeof(float2) ? kFP32 : kFP16);
#define PTC_FUSED(CI, CO)                                                                                          \
  hipLaunchKernelGGL((k_ptc_fused<SA, SL, CI, CO>), grid, block, 0, st, g, in, out, U, recon, (const short*)n->Af[l], \
                     fused_kp(L), oscale, scal, ftz)
  if (L.cin == 1 && L.cout == 1) PTC_FUSED(1, 1);
  else if (L.cin == 1) PTC_FUSED(1, 2);
  else if (L.cout == 1) PTC_FUSED(2, 1);
  else PTC_FUSED(2, 2);
#undef PTC_FUSED
}

// Forward through all layers from act[0].  With train, the two-pass form
// keeps the transported inputs of every layer for the backward pass; else
// each layer is one fused kernel.
template <typename E> void two_pass_layer(qcd_ptc* n, int l, int nb, hipStream_t st) {
  const Geom& g = n->g;
  hipLaunchKernelGGL(k_ptc_transport<E>, dim3(site_blocks_pad(g), nb), dim3(256), 0, st, g, n->L[l],
                     (const float2*)n->act[l], links32(n), recon_of(n, kFP32), (E*)n->X[l]);
  hipLaunchKernelGGL(k_ptc_mix<E>, dim3(n->mix_blocks), dim3(256), 0, st, g, n->L[l], (const E*)n->X[l],
                     (const E*)n->A[l], n->act[l + 1], nb);
}

// (the FP32 mixing mode runs every FP32-activation forward in the two-pass form)
qcd_status forward(qcd_ptc* n, int nb, bool train, hipStream_t st) {
  if (train || n->mix_fp32) {
    qcd_status rc = ensure_two_pass(n);
    if (rc) return rc;
  }
  for (int l = 0; l < n->nlayers; l++) {
    if (n->mix_fp32) {
      two_pass_layer<float>(n, l, nb, st);
    } else if (!train) {
      fused_layer<float2, float2>(n, l, nb, n->act[l], n->act[l + 1], links32(n), 1.0f, nullptr, 0, st);
    } else {
      two_pass_layer<short>(n, l, nb, st);
    }
  }
  return QCD_OK;
}

// One layer's backward from dact[cur]: weight gradient into n->grad, and
// (l > 0) the input gradient into dact[cur ^ 1].
template <typename E> void backward_layer(qcd_ptc* n, int l, int nb, int cur, hipStream_t st) {
  const Geom& g = n->g;
  const PtcLayerDev& L = n->L[l];
  hipLaunchKernelGGL(k_ptc_dout_mix<E>, dim3(site_blocks_pad(g), nb), dim3(256), 0, st, g, L,
                     (const float2*)n->dact[cur], (E*)n->DO);
  hipLaunchKernelGGL(k_ptc_mix_dw<E>, dim3(n->mix_blocks), dim3(256), 0, st, g, L, (const E*)n->DO,
                     (const E*)n->X[l], n->Gp, nb);
  hipLaunchKernelGGL(k_ptc_dw_slices, dim3((L.M * L.K + 63) / 64, kDwSlices), dim3(64), 0, st, L,
                     (const float*)n->Gp, n->mix_blocks * 4, n->dwp);
  hipLaunchKernelGGL(k_ptc_dw_finish, dim3((L.M * L.K + 255) / 256), dim3(256), 0, st, L, (const double*)n->dwp,
                     n->grad + n->woff[l]);
  if (l > 0) {
    hipLaunchKernelGGL(k_ptc_mix_dx<E>, dim3(n->mix_blocks), dim3(256), 0, st, g, L, (const E*)n->DO,
                       (const E*)n->A[l], n->DX, nb);
    hipLaunchKernelGGL(k_ptc_transport_adj, dim3(site_blocks(g), nb), dim3(256), 0, st, g, L, (const float*)n->DX,
                       links32(n), recon_of(n, kFP32), n->dact[cur ^ 1]);
  }
}

// Weight gradient (into n->grad) from the output gradient in dact[0].
void backward(qcd_ptc* n, int nb, hipStream_t st) {
  int cur = 0;
  for (int l = n->nlayers - 1; l >= 0; l--) {
    if (n->mix_fp32) backward_layer<float>(n, l, nb, cur, st);
    else backward_layer<short>(n, l, nb, cur, st);
    if (l > 0) cur ^= 1;
  }
}

// mean over the batch of sums[2b] / sums[2b + 1] (synchronises)
qcd_status read_loss(qcd_ptc* n, int nb, double* loss, hipStream_t st) {
  std::vector<double> h(2 * nb);
  PTC_TRY(hipMemcpyAsync(h.data(), n->sums, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, st));
  PTC_TRY(hipStreamSynchronize(st));
  double tot = 0;
  for (int b = 0; b < nb; b++) tot += h[2 * b] / h[2 * b + 1];
  *loss = tot / nb;
  return QCD_OK;
}

// Loss and gradient of the weights (into n->grad) for the batch in act[0] / target.
qcd_status loss_grad(qcd_ptc* n, int nb, double* loss, hipStream_t st) {
  const Geom& g = n->g;
  qcd_status rc = forward(n, nb, true, st);
  if (rc) return rc;
  const int last = n->nlayers;
  hipLaunchKernelGGL(k_ptc_loss_parts, dim3(site_blocks(g), nb), dim3(256), 0, st, g, (const float2*)n->act[last],
                     (const float2*)n->target, n->partials);
  hipLaunchKernelGGL(k_ptc_loss_finish, dim3(nb), dim3(1024), 0, st, (const double*)n->partials, site_blocks(g), nb,
                     n->sums);
  hipLaunchKernelGGL(k_ptc_dout, dim3(site_blocks(g), nb), dim3(256), 0, st, g, (const float2*)n->act[last],
                     (const float2*)n->target, (const double*)n->sums, nb, n->dact[0]);
  PTC_TRY(hipMemsetAsync(n->grad, 0, n->nweights * sizeof(float2), st));
  backward(n, nb, st);
  PTC_LAUNCHED();
  if (loss) return read_loss(n, nb, loss, st);
  return QCD_OK;
}

// The residual loss (1/B) sum_b |D M r_b - r_b|^2 / |r_b|^2 for the batch in
// act[0], D the Wilson matrix of eq. (1) (FP32 operator on the handle's FP32
// links), and its weight gradient: the output gradient is
// 2 / (B |r_b|^2) D^dag (D M r_b - r_b).  target holds D M r, dact[1] the
// scaled residual before D^dag.
qcd_status loss_grad_residual(qcd_ptc* n, double kappa, int nb, double* loss, hipStream_t st) {
  const Geom& g = n->g;
  const qcd_gauge* G = n->gauge;
  qcd_status rc = forward(n, nb, true, st);
  if (rc) return rc;
  const int last = n->nlayers;
  launch_dslash(kFP32, g, G->tune[kFP32], kOpD, kEpiNone, nb, n->target, n->act[last], G->U[kFP32], kappa, nullptr,
                nullptr, nullptr, 0, st);
  hipLaunchKernelGGL(k_ptc_loss_parts, dim3(site_blocks(g), nb), dim3(256), 0, st, g, (const float2*)n->target,
                     (const float2*)n->act[0], n->partials);
  hipLaunchKernelGGL(k_ptc_loss_finish, dim3(nb), dim3(1024), 0, st, (const double*)n->partials, site_blocks(g), nb,
                     n->sums);
  hipLaunchKernelGGL(k_ptc_dout, dim3(site_blocks(g), nb), dim3(256), 0, st, g, (const float2*)n->target,
                     (const float2*)n->act[0], (const double*)n->sums, nb, n->dact[1]);
  launch_dslash(kFP32, g, G->tune[kFP32], kOpDdag, kEpiNone, nb, n->dact[0], n->dact[1], G->U[kFP32], kappa, nullptr,
                nullptr, nullptr, 0, st);
  PTC_TRY(hipMemsetAsync(n->grad, 0, n->nweights * sizeof(float2), st));
  backward(n, nb, st);
  PTC_LAUNCHED();
  if (loss) return read_loss(n, nb, loss, st);
  return QCD_OK;
}

// Adam on the FP32 master weights from n->grad, then the GEMM operands.
void adam_step(qcd_ptc* n, double lr, hipStream_t st) {
  n->adam_step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)n->adam_step), c2 = 1.0f - powf(b2, (float)n->adam_step);
  const int cnt = (int)(2 * n->nweights);
  hipLaunchKernelGGL(k_adam, dim3((cnt + 255) / 256), dim3(256), 0, st, (float*)n->w, (const float*)n->grad,
                     (float*)n->adam_m, (float*)n->adam_v, cnt, (float)lr, b1, b2, 1e-8f, c1, c2);
  prep_weights(n, st);
}

// Replace one of the handle's buffers by a new one of `bytes`.
qcd_status realloc_buf(qcd_ptc* n, void** p, size_t bytes) {
  void* q = nullptr;
  PTC_TRY(hipMalloc(&q, bytes ? bytes : 256));
  for (auto& a : n->allocs)
    if (a == *p) {
      (void)hipFree(a);
      a = q;
      *p = q;
      return QCD_OK;
    }
  n->allocs.push_back(q);
  *p = q;
  return QCD_OK;
}

qcd_status check_batch(const qcd_ptc* n, int nb) {
  if (!n) return pfail(QCD_ERR_ARG, "null network handle");
  if (nb < 1 || nb > n->max_batch) return pfail(QCD_ERR_ARG, "batch must be in 1..%d", n->max_batch);
  return QCD_OK;
}

}  // namespace

namespace qcd {
// Apply the network to nb native FP16 fields: out = scale * M(in), FP16
// activations and FP16 links (the inner solver's), one fused kernel per
// layer.  Used by the preconditioned inner solver (all launches are
// stream-ordered and capturable); batches whose solver has stopped are
// skipped when scal is given.
// More than max_batch fields are taken max_batch at a time (the hidden
// activations hold max_batch elements).
void ptc_apply_half(qcd_ptc* n, int nb, const void* in, void* out, float scale, int ftz, const Scalars* scal,
                    hipStream_t st) {
  const __half2* U = (const __half2*)n->gauge->U[kFP16];
  const size_t fe = spinor_elems(n->g);
  for (int b0 = 0; b0 < nb; b0 += n->max_batch) {
    const int c = std::min(n->max_batch, nb - b0);
    const __half2* src = (const __half2*)in + b0 * fe;
    for (int l = 0; l < n->nlayers; l++) {
      const bool last = l == n->nlayers - 1;
      __half2* dst = last ? (__half2*)out + b0 * fe : n->act16[l + 1];
      fused_layer<__half2, __half2>(n, l, c, src, dst, U, last ? scale : 1.0f, scal ? scal + b0 : nullptr, ftz, st);
      src = dst;
    }
  }
}
// Largest |M(v_b)| / |v_b| over the nb native FP16 fields v_b (zero fields
// skipped); synchronises.  Returns 0 if every field is zero.
qcd_status ptc_gain(qcd_ptc* n, int nb, const void* in, double* gain, hipStream_t st) {
  const Geom& g = n->g;
  if (!n->gauge->U[kFP16]) return pfail(QCD_ERR_ARG, "the gauge handle holds no FP16 links");
  double best = 0;
  std::vector<double> h(2 * n->max_batch);
  for (int b0 = 0; b0 < nb; b0 += n->max_batch) {  // max_batch fields at a time
    const int c = std::min(n->max_batch, nb - b0);
    hipLaunchKernelGGL(k_h2f, dim3(site_blocks(g), c), dim3(256), 0, st, g,
                       (const __half2*)in + (size_t)b0 * spinor_elems(g), n->act[0], 1.0f);
    qcd_status rc = forward(n, c, false, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_ptc_norms, dim3(site_blocks(g), c), dim3(256), 0, st, g, (const float2*)n->act[0],
                       (const float2*)n->act[n->nlayers], n->partials);
    hipLaunchKernelGGL(k_ptc_loss_finish, dim3(c), dim3(1024), 0, st, (const double*)n->partials, site_blocks(g), c,
                       n->sums);
    PTC_LAUNCHED();
    PTC_TRY(hipMemcpyAsync(h.data(), n->sums, 2 * c * sizeof(double), hipMemcpyDeviceToHost, st));
    PTC_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < c; b++)
      if (h[2 * b] > 0 && std::isfinite(h[2 * b + 1])) best = std::max(best, std::sqrt(h[2 * b + 1] / h[2 * b]));
      else if (h[2 * b] > 0) return pfail(QCD_ERR_NONFINITE, "network output is not finite");
  }
  *gain = best;
  return QCD_OK;
}
int ptc_max_batch(const qcd_ptc* n) { return n->max_batch; }
const qcd_gauge* ptc_gauge(const qcd_ptc* n) { return n->gauge; }
}  // namespace qcd

extern "C" {

qcd_status qcd_ptc_free(qcd_ptc* n) {
  if (!n) return QCD_OK;
  for (void* p : n->allocs) (void)hipFree(p);
  delete n;
  return QCD_OK;
}

qcd_status qcd_ptc_create(qcd_ptc** out, const qcd_gauge* gauge, int nlayers, const int* channels, int max_batch,
                          void* stream) {
  if (!out || !gauge || !channels) return pfail(QCD_ERR_ARG, "null argument");
  if (nlayers < 1 || nlayers > kPtcMaxLayers) return pfail(QCD_ERR_ARG, "nlayers must be in 1..%d", kPtcMaxLayers);
  if (max_batch < 1 || max_batch > kMaxRhs) return pfail(QCD_ERR_ARG, "max_batch must be in 1..%d", kMaxRhs);
  if (!gauge->U[kFP32]) return pfail(QCD_ERR_ARG, "the network needs the gauge handle's FP32 links");
  for (int l = 0; l <= nlayers; l++)
    if (channels[l] < 1 || channels[l] > 2) return pfail(QCD_ERR_UNSUPPORTED, "channels must be 1 or 2 per layer");
  if (channels[0] != 1 || channels[nlayers] != 1)
    return pfail(QCD_ERR_ARG, "the network maps one spinor field to one spinor field");
  qcd_ptc* n = new qcd_ptc();
  n->gauge = gauge;
  n->g = gauge->g;
  n->nlayers = nlayers;
  n->max_batch = max_batch;
  n->nweights = 0;
  int maxKp = 16;
  for (int l = 0; l <= nlayers; l++) n->channels[l] = channels[l];
  for (int l = 0; l < nlayers; l++) {
    PtcLayerDev& L = n->L[l];
    L.cin = channels[l];
    L.cout = channels[l + 1];
    L.K = 9 * L.cin * 4;
    L.M = L.cout * 4;
    L.Kp = ((2 * L.K + 15) / 16) * 16;
    n->woff[l] = n->nweights;
    n->nweights += (size_t)9 * L.cout * L.cin * 16;
    maxKp = std::max(maxKp, L.Kp);
  }
  const Geom& g = n->g;
  n->mix_blocks = 1024;
  qcd_status rc = QCD_OK;
#define PTC_ALLOC(ptr, bytes) \
  if (rc == QCD_OK) rc = alloc(n, (void**)&(ptr), (bytes))
  PTC_ALLOC(n->w, n->nweights * sizeof(float2));
  PTC_ALLOC(n->grad, n->nweights * sizeof(float2));
  PTC_ALLOC(n->adam_m, n->nweights * sizeof(float2));
  PTC_ALLOC(n->adam_v, n->nweights * sizeof(float2));
  for (int l = 0; l < nlayers; l++) {
    PTC_ALLOC(n->A[l], 16 * (size_t)n->L[l].Kp * sizeof(short));
    PTC_ALLOC(n->Af[l], 16 * (size_t)fused_kp(n->L[l]) * sizeof(short));
  }
  for (int l = 0; l <= nlayers; l++) PTC_ALLOC(n->act[l], fields_bytes(g, (size_t)max_batch * channels[l]));
  // act16[0] and act16[nlayers] hold the input and output of qcd_ptc_apply_prec in FP16
  for (int l = 0; l <= nlayers; l++)
    PTC_ALLOC(n->act16[l], (size_t)max_batch * channels[l] * spinor_elems(g) * sizeof(__half2));
  PTC_ALLOC(n->Gp, (size_t)n->mix_blocks * 4 * 16 * maxKp * sizeof(float));
  size_t max_mk = 0;
  for (int l = 0; l < nlayers; l++) max_mk = std::max(max_mk, (size_t)n->L[l].M * n->L[l].K);
  PTC_ALLOC(n->dwp, (size_t)kDwSlices * max_mk * 4 * sizeof(double));
  PTC_ALLOC(n->partials, (size_t)max_batch * site_blocks(g) * 2 * sizeof(double));
  PTC_ALLOC(n->sums, (size_t)max_batch * 2 * sizeof(double));
#undef PTC_ALLOC
  hipStream_t st = (hipStream_t)stream;
  if (rc == QCD_OK) {
    // activations of padding sites are never written: clear once so they stay finite
    for (int l = 0; l <= nlayers; l++)
      (void)hipMemsetAsync(n->act[l], 0, fields_bytes(g, (size_t)max_batch * channels[l]), st);
    for (int l = 0; l <= nlayers; l++)
      (void)hipMemsetAsync(n->act16[l], 0, (size_t)max_batch * channels[l] * spinor_elems(g) * sizeof(__half2), st);
    (void)hipMemsetAsync(n->w, 0, n->nweights * sizeof(float2), st);
    (void)hipMemsetAsync(n->adam_m, 0, n->nweights * sizeof(float2), st);
    (void)hipMemsetAsync(n->adam_v, 0, n->nweights * sizeof(float2), st);
    prep_weights(n, st);
    if (hipStreamSynchronize(st) != hipSuccess) rc = pfail(QCD_ERR_HIP, "synchronise failed");
  }
  if (rc != QCD_OK) {
    qcd_ptc_free(n);
    return rc;
  }
  *out = n;
  return QCD_OK;
}

size_t qcd_ptc_num_weights(const qcd_ptc* n) { return n ? n->nweights : 0; }

qcd_status qcd_ptc_set_weights(qcd_ptc* n, const double* w_host, void* stream) {
  if (!n || !w_host) return pfail(QCD_ERR_ARG, "null argument");
  std::vector<float2> h(n->nweights);
  for (size_t i = 0; i < n->nweights; i++) h[i] = make_float2((float)w_host[2 * i], (float)w_host[2 * i + 1]);
  hipStream_t st = (hipStream_t)stream;
  PTC_TRY(hipMemcpyAsync(n->w, h.data(), n->nweights * sizeof(float2), hipMemcpyHostToDevice, st));
  PTC_TRY(hipMemsetAsync(n->adam_m, 0, n->nweights * sizeof(float2), st));
  PTC_TRY(hipMemsetAsync(n->adam_v, 0, n->nweights * sizeof(float2), st));
  n->adam_step = 0;
  prep_weights(n, st);
  PTC_LAUNCHED();
  PTC_TRY(hipStreamSynchronize(st));
  return QCD_OK;
}

qcd_status qcd_ptc_get_weights(const qcd_ptc* n, double* w_host, void* stream) {
  if (!n || !w_host) return pfail(QCD_ERR_ARG, "null argument");
  std::vector<float2> h(n->nweights);
  hipStream_t st = (hipStream_t)stream;
  PTC_TRY(hipMemcpyAsync(h.data(), n->w, n->nweights * sizeof(float2), hipMemcpyDeviceToHost, st));
  PTC_TRY(hipStreamSynchronize(st));
  for (size_t i = 0; i < n->nweights; i++) {
    w_host[2 * i] = h[i].x;
    w_host[2 * i + 1] = h[i].y;
  }
  return QCD_OK;
}

qcd_status qcd_ptc_apply(qcd_ptc* n, int nbatch, void* out_dev, const void* in_dev, void* stream) {
  qcd_status rc = check_batch(n, nbatch);
  if (rc) return rc;
  if (!out_dev || !in_dev) return pfail(QCD_ERR_ARG, "null vector");
  hipStream_t st = (hipStream_t)stream;
  launch_pack_spinor(n->g, kFP32, nbatch, n->act[0], (const double*)in_dev, 1.0, 0, nullptr, st);
  if ((rc = forward(n, nbatch, false, st))) return rc;
  launch_unpack_spinor(n->g, kFP32, nbatch, (double*)out_dev, n->act[n->nlayers], nullptr, 1.0, st);
  PTC_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_ptc_apply_prec(qcd_ptc* n, qcd_prec prec, int nbatch, void* out_dev, const void* in_dev,
                              void* stream) {
  if (prec == QCD_FP32) return qcd_ptc_apply(n, nbatch, out_dev, in_dev, stream);
  if (prec != QCD_FP16) return pfail(QCD_ERR_ARG, "the network applies in FP32 or FP16");
  qcd_status rc = check_batch(n, nbatch);
  if (rc) return rc;
  if (!out_dev || !in_dev) return pfail(QCD_ERR_ARG, "null vector");
  if (!n->gauge->U[kFP16]) return pfail(QCD_ERR_ARG, "the gauge handle holds no FP16 links");
  hipStream_t st = (hipStream_t)stream;
  launch_pack_spinor(n->g, kFP16, nbatch, n->act16[0], (const double*)in_dev, 1.0, 0, nullptr, st);
  ptc_apply_half(n, nbatch, n->act16[0], n->act16[n->nlayers], 1.0f, 0, nullptr, st);
  launch_unpack_spinor(n->g, kFP16, nbatch, (double*)out_dev, n->act16[n->nlayers], nullptr, 1.0, st);
  PTC_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_ptc_loss_grad(qcd_ptc* n, int nbatch, const void* r_dev, const void* e_dev, double* loss,
                             double* grad_host, void* stream) {
  qcd_status rc = check_batch(n, nbatch);
  if (rc) return rc;
  if (!r_dev || !e_dev) return pfail(QCD_ERR_ARG, "null vector");
  if ((rc = ensure_two_pass(n))) return rc;
  hipStream_t st = (hipStream_t)stream;
  launch_pack_spinor(n->g, kFP32, nbatch, n->act[0], (const double*)r_dev, 1.0, 0, nullptr, st);
  launch_pack_spinor(n->g, kFP32, nbatch, n->target, (const double*)e_dev, 1.0, 0, nullptr, st);
  if ((rc = loss_grad(n, nbatch, loss, st))) return rc;
  if (grad_host) {
    std::vector<float2> h(n->nweights);
    PTC_TRY(hipMemcpyAsync(h.data(), n->grad, n->nweights * sizeof(float2), hipMemcpyDeviceToHost, st));
    PTC_TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < n->nweights; i++) {
      grad_host[2 * i] = h[i].x;
      grad_host[2 * i + 1] = h[i].y;
    }
  }
  return QCD_OK;
}

qcd_status qcd_ptc_train_step(qcd_ptc* n, int nbatch, const void* r_dev, const void* e_dev, double lr, double* loss,
                              void* stream) {
  qcd_status rc = qcd_ptc_loss_grad(n, nbatch, r_dev, e_dev, loss, nullptr, stream);
  if (rc) return rc;
  adam_step(n, lr, (hipStream_t)stream);
  PTC_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_ptc_loss_grad_residual(qcd_ptc* n, double kappa, int nbatch, const void* r_dev, double* loss,
                                      double* grad_host, void* stream) {
  qcd_status rc = check_batch(n, nbatch);
  if (rc) return rc;
  if (!r_dev) return pfail(QCD_ERR_ARG, "null vector");
  if (!(kappa > 0) || !std::isfinite(kappa)) return pfail(QCD_ERR_ARG, "kappa must be positive and finite");
  hipStream_t st = (hipStream_t)stream;
  launch_pack_spinor(n->g, kFP32, nbatch, n->act[0], (const double*)r_dev, 1.0, 0, nullptr, st);
  if ((rc = loss_grad_residual(n, kappa, nbatch, loss, st))) return rc;
  if (grad_host) {
    std::vector<float2> h(n->nweights);
    PTC_TRY(hipMemcpyAsync(h.data(), n->grad, n->nweights * sizeof(float2), hipMemcpyDeviceToHost, st));
    PTC_TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < n->nweights; i++) {
      grad_host[2 * i] = h[i].x;
      grad_host[2 * i + 1] = h[i].y;
    }
  }
  return QCD_OK;
}

qcd_status qcd_ptc_train_step_residual(qcd_ptc* n, double kappa, int nbatch, const void* r_dev, double lr,
                                       double* loss, void* stream) {
  qcd_status rc = qcd_ptc_loss_grad_residual(n, kappa, nbatch, r_dev, loss, nullptr, stream);
  if (rc) return rc;
  adam_step(n, lr, (hipStream_t)stream);
  PTC_LAUNCHED();
  return QCD_OK;
}

qcd_status qcd_ptc_set_mixing(qcd_ptc* n, qcd_prec prec, void* stream) {
  if (!n) return pfail(QCD_ERR_ARG, "null network handle");
  if (prec != QCD_BF16 && prec != QCD_FP32) return pfail(QCD_ERR_ARG, "the mixing runs in BF16 or FP32");
  const int want = prec == QCD_FP32;
  if (want == n->mix_fp32) return QCD_OK;
  hipStream_t st = (hipStream_t)stream;
  PTC_TRY(hipStreamSynchronize(st));  // no launch may still read the old buffers
  const size_t es = want ? sizeof(float) : sizeof(short);
  const size_t N = gemm_rows(n->g);
  const int maxKp = max_kp(n);
  qcd_status rc = QCD_OK;
  for (int l = 0; l < n->nlayers && rc == QCD_OK; l++) {
    rc = realloc_buf(n, &n->A[l], 16 * (size_t)n->L[l].Kp * es);
    if (rc == QCD_OK && n->two_pass_ready)  // else they are made at the new width on first use
      rc = realloc_buf(n, &n->X[l], (size_t)n->max_batch * N * (l == 0 ? maxKp : n->L[l].Kp) * es);
  }
  if (rc == QCD_OK && n->two_pass_ready) rc = realloc_buf(n, &n->DO, (size_t)n->max_batch * N * 16 * es);
  if (rc) return rc;
  n->mix_fp32 = want;
  prep_weights(n, st);
  PTC_LAUNCHED();
  PTC_TRY(hipStreamSynchronize(st));
  return QCD_OK;
}

qcd_status qcd_ptc_set_gauge(qcd_ptc* n, const qcd_gauge* gauge) {
  if (!n || !gauge) return pfail(QCD_ERR_ARG, "null argument");
  if (!gauge->U[kFP32]) return pfail(QCD_ERR_ARG, "the network needs the gauge handle's FP32 links");
  for (int mu = 0; mu < 4; mu++)
    if (gauge->dims[mu] != n->gauge->dims[mu]) return pfail(QCD_ERR_ARG, "lattice extents differ");
  n->gauge = gauge;
  return QCD_OK;
}

qcd_status qcd_ptc_init_neumann(qcd_ptc* n, double kappa, void* stream) {
  if (!n) return pfail(QCD_ERR_ARG, "null network handle");
  const int want[4] = {1, 2, 2, 1};
  if (n->nlayers != 3 || memcmp(n->channels, want, sizeof want) != 0)
    return pfail(QCD_ERR_UNSUPPORTED, "the Neumann form is defined for channels 1, 2, 2, 1");
  // Spin matrices of the hops of kappa H: path +mu carries kappa (1 - gamma_mu),
  // path -mu kappa (1 + gamma_mu), in the Dirac basis of the Wilson kernel
  // (gamma_1 as printed in Sec. 2; gamma_4 = diag(1, 1, -1, -1)).
  typedef std::complex<double> C;
  const C I(0, 1);
  C gam[4][4][4] = {};
  gam[0][0][3] = -I; gam[0][1][2] = -I; gam[0][2][1] = I; gam[0][3][0] = I;
  gam[1][0][3] = -1; gam[1][1][2] = 1;  gam[1][2][1] = 1; gam[1][3][0] = -1;
  gam[2][0][2] = -I; gam[2][1][3] = I;  gam[2][2][0] = I; gam[2][3][1] = -I;
  gam[3][0][0] = 1;  gam[3][1][1] = 1;  gam[3][2][2] = -1; gam[3][3][3] = -1;
  std::vector<double> w(2 * n->nweights, 0.0);
  // weight W[p][j][i][s'][s] of layer l
  auto put = [&](int l, int p, int j, int i, int sp, int sv, C v) {
    const PtcLayerDev& L = n->L[l];
    const size_t k = n->woff[l] + ((((size_t)p * L.cout + j) * L.cin + i) * 4 + sp) * 4 + sv;
    w[2 * k] += v.real();
    w[2 * k + 1] += v.imag();
  };
  auto ident = [&](int l, int j, int i) {
    for (int s = 0; s < 4; s++) put(l, 0, j, i, s, s, 1.0);
  };
  auto hop = [&](int l, int j, int i) {  // out_j += kappa H in_i
    for (int mu = 0; mu < 4; mu++)
      for (int sp = 0; sp < 4; sp++)
        for (int sv = 0; sv < 4; sv++) {
          const C d = sp == sv ? 1.0 : 0.0;
          put(l, 1 + 2 * mu, j, i, sp, sv, kappa * (d - gam[mu][sp][sv]));
          put(l, 2 + 2 * mu, j, i, sp, sv, kappa * (d + gam[mu][sp][sv]));
        }
  };
  // layer 0: (psi, kH psi); layer 1: (c0 + c1, kH (c0 + c1)); layer 2: c0 + kH c1
  // => M = (1 + kH)(1 + (kH)^2) = sum_{k <= 3} (kappa H)^k
  ident(0, 0, 0); hop(0, 1, 0);
  ident(1, 0, 0); ident(1, 0, 1); hop(1, 1, 0); hop(1, 1, 1);
  ident(2, 0, 0); hop(2, 0, 1);
  return qcd_ptc_set_weights(n, w.data(), stream);
}

}  // extern "C"
