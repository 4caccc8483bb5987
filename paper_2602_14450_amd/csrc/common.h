// Shared device-side definitions for the Wilson-Dirac solver library:
// complex arithmetic, storage formats, the native (checkerboarded,
// wavefront-blocked) field layout, and deterministic block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace qcd {

// ---------------------------------------------------------------------------
// Complex arithmetic in the compute type T (float or double).
template <typename T> struct cx {
  T re, im;
  __device__ __host__ cx() {}
  __device__ __host__ cx(T r, T i) : re(r), im(i) {}
};
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.im, a.re}; }   //  i a
template <typename T> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }  // -i a
template <typename T> __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// Storage formats.  A stored complex number is one element of S; the
// arithmetic type is Traits<S>::T.  FP16 storage packs (re, im) into one
// 32-bit __half2 word; arithmetic on it is FP32.
template <typename S> struct Traits;
template <> struct Traits<double2> {
  using T = double;
  static __device__ __forceinline__ cx<double> load(const double2* p) { double2 v = *p; return {v.x, v.y}; }
  static __device__ __forceinline__ double2 pack(cx<double> v, int) { return make_double2(v.re, v.im); }
};
template <> struct Traits<float2> {
  using T = float;
  static __device__ __forceinline__ cx<float> load(const float2* p) { float2 v = *p; return {v.x, v.y}; }
  static __device__ __forceinline__ float2 pack(cx<float> v, int) { return make_float2(v.re, v.im); }
};
// Smallest normal binary16 magnitude, 2^-14.
constexpr float kHalfMinNormal = 6.103515625e-05f;
template <> struct Traits<__half2> {
  using T = float;
  static __device__ __forceinline__ cx<float> load(const __half2* p) {
    float2 v = __half22float2(*p);
    return {v.x, v.y};
  }
  // Round to nearest even; with ftz set, a result below the smallest normal
  // binary16 magnitude is replaced by a zero of the same sign.
  static __device__ __forceinline__ __half2 pack(cx<float> v, int ftz) {
    __half2 h = __floats2half2_rn(v.re, v.im);
    if (ftz) {
      float2 f = __half22float2(h);
      if (fabsf(f.x) < kHalfMinNormal) f.x = copysignf(0.0f, f.x);
      if (fabsf(f.y) < kHalfMinNormal) f.y = copysignf(0.0f, f.y);
      h = __floats2half2_rn(f.x, f.y);
    }
    return h;
  }
};

// BF16 storage (Table 1: 8 exponent bits, 7 fraction bits): one complex is
// two bfloat16 halves of a 32-bit word, like FP16; arithmetic on it is FP32.
struct alignas(4) bf2 {
  __bf16 x, y;
};
constexpr float kBf16MinNormal = 1.17549435e-38f;  // 2^-126
template <> struct Traits<bf2> {
  using T = float;
  static __device__ __forceinline__ cx<float> load(const bf2* p) {
    const bf2 v = *p;
    return {(float)v.x, (float)v.y};
  }
  // Round to nearest even; with ftz set, a result below 2^-126 in magnitude
  // is replaced by a zero of the same sign.
  static __device__ __forceinline__ bf2 pack(cx<float> v, int ftz) {
    bf2 b{(__bf16)v.re, (__bf16)v.im};
    if (ftz) {
      if (fabsf((float)b.x) < kBf16MinNormal) b.x = (__bf16)copysignf(0.0f, v.re);
      if (fabsf((float)b.y) < kBf16MinNormal) b.y = (__bf16)copysignf(0.0f, v.im);
    }
    return b;
  }
};

// FP64 value -> stored format: one round-to-nearest-even conversion
// (for FP16 the compiler emits a correctly rounded FP64 -> FP16 sequence).
template <typename S> __device__ __forceinline__ S pack_from_double(double re, double im, int ftz);
template <> __device__ __forceinline__ double2 pack_from_double<double2>(double re, double im, int) { return make_double2(re, im); }
template <> __device__ __forceinline__ float2 pack_from_double<float2>(double re, double im, int) {
  return make_float2((float)re, (float)im);
}
// FP64 -> BF16 in one rounding (the compiler rounds to FP32 with the
// round-to-odd rule first, which makes the second rounding exact).
template <> __device__ __forceinline__ bf2 pack_from_double<bf2>(double re, double im, int ftz) {
  bf2 b{(__bf16)re, (__bf16)im};
  if (ftz) {
    if (fabsf((float)b.x) < kBf16MinNormal) b.x = (__bf16)copysignf(0.0f, (float)re);
    if (fabsf((float)b.y) < kBf16MinNormal) b.y = (__bf16)copysignf(0.0f, (float)im);
  }
  return b;
}
template <> __device__ __forceinline__ __half2 pack_from_double<__half2>(double re, double im, int ftz) {
  __half2 h = __half2{_Float16_2{static_cast<_Float16>(re), static_cast<_Float16>(im)}};
  if (ftz) {
    float2 f = __half22float2(h);
    if (fabsf(f.x) < kHalfMinNormal) f.x = copysignf(0.0f, f.x);
    if (fabsf(f.y) < kHalfMinNormal) f.y = copysignf(0.0f, f.y);
    h = __floats2half2_rn(f.x, f.y);
  }
  return h;
}

// ---------------------------------------------------------------------------
// Unsigned division by a run-time constant d >= 1 for n < 2^31 (round-up
// multiplier method of Granlund & Montgomery, PLDI 1994).
struct FastDiv {
  uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) s++;
  f.s = s;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return (__umulhi(n, f.m) + n) >> f.s; }

// ---------------------------------------------------------------------------
// Native layout.
//
// Sites are split by parity p = (x+y+z+t) & 1.  Within a parity, site
// (x,y,z,t) has half index h = (x>>1) + Lx/2*(y + Ly*(z + Lz*t)).  Half
// indices are grouped in blocks of 64 (one wavefront).  Each block stores its
// complex components in 16-byte granules: with C = 16 / sizeof(stored
// complex) components per granule (4 for FP16 and BF16, 2 for FP32, 1 for FP64),
// granule row j holds components [jC, jC+C) of the 64 sites, lane-major, so
// that lane i of a wave reading row j issues one 16-byte load at
// (block*12*64 + j*64*C + i*C) and the wave reads one contiguous 1 KB
// segment.  A spinor block holds 12 components (spin-major, colour fastest);
// a link block (per direction and parity) holds the 9 entries U[a][b]
// (row-major), the first F = (9/C)*C in full granule rows and the rest in
// rows of one component per lane.
struct Geom {
  int L[4];
  int Lxh;         // Lx / 2
  int Vh;          // sites per parity
  int nb;          // 64-site blocks per parity
  int sy, sz, st;  // half-index strides of y, z, t
  FastDiv dx, dy, dz, dnb;
  int npar;        // parities a field holds: 2 (full field, even then odd) or 1 (one parity, indexed as parity 0)
};

inline Geom make_geom(const int dims[4]) {
  Geom g;
  for (int i = 0; i < 4; i++) g.L[i] = dims[i];
  g.Lxh = dims[0] / 2;
  g.Vh = g.Lxh * dims[1] * dims[2] * dims[3];
  g.nb = (g.Vh + 63) / 64;
  g.sy = g.Lxh;
  g.sz = g.Lxh * dims[1];
  g.st = g.Lxh * dims[1] * dims[2];
  g.dx = make_fastdiv(g.Lxh);
  g.dy = make_fastdiv(dims[1]);
  g.dz = make_fastdiv(dims[2]);
  g.dnb = make_fastdiv(g.nb);
  g.npar = 2;
  return g;
}
// The same lattice seen through fields of one parity (the even-odd solver's
// vectors): streaming kernels then run over Vh sites, indexed as parity 0.
inline Geom half_geom(const Geom& g) {
  Geom h = g;
  h.npar = 1;
  return h;
}

// Elements (stored complex numbers) of one full native spinor / link field.
// A link field stores ne complex entries per link: 9 (the full matrix) or 6
// (rows 0 and 1 of an SU(3) matrix; row 2 is rebuilt as conj(row0 x row1)).
__host__ __device__ inline size_t spinor_elems(const Geom& g) { return (size_t)g.npar * g.nb * 12 * 64; }
__host__ __device__ inline size_t link_elems(const Geom& g, int ne = 9) { return (size_t)4 * 2 * g.nb * ne * 64; }

template <typename S> struct Lay {
  static constexpr int C = 16 / (int)sizeof(S);  // components per granule
  static constexpr int G = 12 / C;               // granule rows of a spinor block
  static constexpr int F = (9 / C) * C;          // link entries in full granule rows
  struct alignas(16) Gran { S s[C]; };
};
// Link block of NE entries: the first F in granule rows, the remaining TAIL
// either as one plane per entry (NE = 9) or packed per lane (NE = 6).
template <typename S, int NE> struct LkLay {
  static constexpr int C = Lay<S>::C;
  static constexpr int F = (NE / C) * C;
  static constexpr int TAIL = NE - F;
};

// Store of a 16-byte granule of the Wilson operator's output (never read by
// the launch that writes it), marked non-temporal so that it streams through
// the L2 instead of displacing neighbour spinors and links that other blocks
// still have to read (5% on the FP16 operator at 32^3 x 64).
// QCD_STREAM_HINTS=0 builds the same kernels with plain loads and stores
// (the hints change timing only; the outputs of the two builds are compared
// bit for bit).
#ifndef QCD_STREAM_HINTS
#define QCD_STREAM_HINTS 1
#endif
template <typename Gr> __device__ __forceinline__ void store_stream(Gr* p, const Gr& v) {
  static_assert(sizeof(Gr) == 16, "granules are 16 bytes");
#if QCD_STREAM_HINTS
  using V = unsigned int __attribute__((ext_vector_type(4)));
  __builtin_nontemporal_store(__builtin_bit_cast(V, v), reinterpret_cast<V*>(p));
#else
  *p = v;
#endif
}
// Load of a 16-byte granule that the launch reads once (the one-parity
// operator's centre and the epilogues' auxiliary fields), marked non-temporal.
template <typename Gr> __device__ __forceinline__ Gr load_stream(const Gr* p) {
  static_assert(sizeof(Gr) == 16, "granules are 16 bytes");
#if QCD_STREAM_HINTS
  using V = unsigned int __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(Gr, __builtin_nontemporal_load(reinterpret_cast<const V*>(p)));
#else
  return *p;
#endif
}

__device__ __forceinline__ size_t sp_block(const Geom& g, int par, int h) {
  return (size_t)(par * g.nb + (h >> 6)) * (12 * 64);
}
template <int NE = 9> __device__ __forceinline__ size_t lk_block(const Geom& g, int mu, int par, int h) {
  return (size_t)((mu * 2 + par) * g.nb + (h >> 6)) * (NE * 64);
}
// element offset of spinor component k of lane `lane` within its block
template <typename S> __device__ __forceinline__ int sp_off(int k, int lane) {
  constexpr int C = Lay<S>::C;
  return (k / C) * 64 * C + lane * C + (k % C);
}
template <typename S, int NE = 9> __device__ __forceinline__ int lk_off(int k, int lane) {
  constexpr int C = Lay<S>::C, F = LkLay<S, NE>::F, TAIL = LkLay<S, NE>::TAIL;
  if (k < F) return (k / C) * 64 * C + lane * C + (k % C);
  return NE == 9 ? F * 64 + (k - F) * 64 + lane : F * 64 + lane * TAIL + (k - F);
}

// Row 2 of an SU(3) matrix from rows 0 and 1: u[6..8] = conj(row0 x row1)
// (unit rows orthogonal to both, with the phase that makes det = 1).
template <typename T> __device__ __forceinline__ void su3_third_row(cx<T> (&u)[9]) {
  const cx<T> a = u[1] * u[5] - u[2] * u[4];
  const cx<T> b = u[2] * u[3] - u[0] * u[5];
  const cx<T> c = u[0] * u[4] - u[1] * u[3];
  u[6] = cx<T>(a.re, -a.im);
  u[7] = cx<T>(b.re, -b.im);
  u[8] = cx<T>(c.re, -c.im);
}

// The link U_mu at (par, h) in either storage form (recon != 0: 6 entries).
template <typename S>
__device__ __forceinline__ void load_link_any(const Geom& g, const S* __restrict__ U, int recon, int mu, int par,
                                              int h, cx<typename Traits<S>::T> (&u)[9]) {
  const int lane = h & 63;
  if (recon) {
    const S* b = U + lk_block<6>(g, mu, par, h);
#pragma unroll
    for (int k = 0; k < 6; k++) u[k] = Traits<S>::load(b + lk_off<S, 6>(k, lane));
    su3_third_row(u);
  } else {
    const S* b = U + lk_block<9>(g, mu, par, h);
#pragma unroll
    for (int k = 0; k < 9; k++) u[k] = Traits<S>::load(b + lk_off<S, 9>(k, lane));
  }
}

struct Coord { int x, y, z, t; };
__device__ __forceinline__ Coord decode(const Geom& g, int par, int h) {
  uint32_t r1 = fdiv((uint32_t)h, g.dx);
  int xh = h - (int)r1 * g.Lxh;
  uint32_t r2 = fdiv(r1, g.dy);
  int y = (int)r1 - (int)r2 * g.L[1];
  uint32_t r3 = fdiv(r2, g.dz);
  int z = (int)r2 - (int)r3 * g.L[2];
  int t = (int)r3;
  int x = 2 * xh + ((par + y + z + t) & 1);
  return {x, y, z, t};
}

// Site-level access to a native spinor (used by the site-ordered kernels).
template <typename S>
__device__ __forceinline__ void load_site(const S* __restrict__ base, const Geom& g, int par, int h,
                                          cx<typename Traits<S>::T> (&f)[12]) {
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C;
  const S* b = base + sp_block(g, par, h);
  const int lane = h & 63;
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++) {
    const Gr v = *reinterpret_cast<const Gr*>(b + j * 64 * C + lane * C);
#pragma unroll
    for (int c = 0; c < C; c++) f[j * C + c] = Traits<S>::load(&v.s[c]);
  }
}
// load_site with non-temporal loads (fields a launch reads once).
template <typename S>
__device__ __forceinline__ void load_site_stream(const S* __restrict__ base, const Geom& g, int par, int h,
                                                 cx<typename Traits<S>::T> (&f)[12]) {
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C;
  const S* b = base + sp_block(g, par, h);
  const int lane = h & 63;
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++) {
    const Gr v = load_stream(reinterpret_cast<const Gr*>(b + j * 64 * C + lane * C));
#pragma unroll
    for (int c = 0; c < C; c++) f[j * C + c] = Traits<S>::load(&v.s[c]);
  }
}
template <typename S>
__device__ __forceinline__ void store_site(S* __restrict__ base, const Geom& g, int par, int h,
                                           const cx<typename Traits<S>::T> (&f)[12], int ftz) {
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C;
  S* b = base + sp_block(g, par, h);
  const int lane = h & 63;
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++) {
    Gr v;
#pragma unroll
    for (int c = 0; c < C; c++) v.s[c] = Traits<S>::pack(f[j * C + c], ftz);
    *reinterpret_cast<Gr*>(b + j * 64 * C + lane * C) = v;
  }
}

// Flat granule view of a native spinor: granule e lies in 64-site block
// e / (768/C), lane (e % (768/C)) % 64.  Padding sites of the last block of
// each parity are skipped.
template <typename S> __device__ __forceinline__ bool gran_valid(const Geom& g, size_t e) {
  constexpr int PER = 768 / Lay<S>::C;
  const uint32_t blk = (uint32_t)(e / PER);
  const int lane = (int)(e % PER) & 63;
  const uint32_t b = blk - fdiv(blk, g.dnb) * (uint32_t)g.nb;
  return b != (uint32_t)(g.nb - 1) || lane < g.Vh - (g.nb - 1) * 64;
}
template <typename S> __host__ __device__ inline size_t spinor_granules(const Geom& g) { return spinor_elems(g) / Lay<S>::C; }

// ---------------------------------------------------------------------------
// Deterministic reductions.  Each thread holds NV FP64 values; the block
// sums them in a fixed tree order and thread 0 writes them to
// partials[blockIdx.x * NV + i].  A single-block finish kernel later sums
// the per-block rows in index order, so results do not depend on timing.
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* partials, int row) {
  __shared__ double red[NV][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; i++) {
    double a = v[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) red[i][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) {
      double s = 0;
      for (int w = 0; w < nw; w++) s += red[i][w];
      partials[(size_t)row * NV + i] = s;
    }
  }
}

// Per-right-hand-side block reduction for blocks whose lanes interleave T
// right-hand sides (lane = site * T + r): lane groups are reduced separately
// and value i of right-hand side r goes to partials[(r0 + r) * rstride + row) * NV + i].
template <int NV, int T>
__device__ __forceinline__ void block_reduce_store_T(double (&v)[NV], double* partials, int r0, int rstride, int row) {
  __shared__ double red[NV][T][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; i++) {
    double a = v[i];
#pragma unroll
    for (int off = 32; off >= T; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane < T) red[i][lane][wid] = a;
  }
  __syncthreads();
  if ((int)threadIdx.x < T) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) {
      double s = 0;
      for (int w = 0; w < nw; w++) s += red[i][threadIdx.x][w];
      partials[((size_t)(r0 + threadIdx.x) * rstride + row) * NV + i] = s;
    }
  }
}

// Sum rows [0, nrows) of partials[nrows][NV] in one block, fixed order.
// Result is valid in out[] on thread 0 after the call.
template <int NV>
__device__ __forceinline__ void finish_sum(const double* partials, int nrows, double (&out)[NV]) {
  __shared__ double red[NV][1024 / 64];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; i++) acc[i] = 0;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
#pragma unroll
    for (int i = 0; i < NV; i++) acc[i] += partials[(size_t)r * NV + i];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; i++) {
    double a = acc[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) red[i][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) {
      double s = 0;
      for (int w = 0; w < nw; w++) s += red[i][w];
      out[i] = s;
    }
  }
}

}  // namespace qcd
