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

// FP64 value -> stored format: one round-to-nearest-even conversion
// (for FP16 the compiler emits a correctly rounded FP64 -> FP16 sequence).
template <typename S> __device__ __forceinline__ S pack_from_double(double re, double im, int ftz);
template <> __device__ __forceinline__ double2 pack_from_double<double2>(double re, double im, int) { return make_double2(re, im); }
template <> __device__ __forceinline__ float2 pack_from_double<float2>(double re, double im, int) {
  return make_float2((float)re, (float)im);
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
// indices are grouped in blocks of 64 (one wavefront).  A spinor stores, for
// each block, its 12 complex components (spin-major, colour fastest) as 12
// runs of 64 consecutive elements, so that lane i of a wave reading
// component k of block b touches element ((p*nb + b)*12 + k)*64 + i:
// every wave-wide access is one contiguous segment.  Links are stored the
// same way per direction: element (((mu*2 + p)*nb + b)*9 + 3a + c)*64 + i.
struct Geom {
  int L[4];
  int Lxh;         // Lx / 2
  int Vh;          // sites per parity
  int nb;          // 64-site blocks per parity
  int sy, sz, st;  // half-index strides of y, z, t
  FastDiv dx, dy, dz;
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
  return g;
}

// Elements of one full native spinor (both parities, padding included).
inline size_t spinor_elems(const Geom& g) { return (size_t)2 * g.nb * 12 * 64; }
inline size_t link_elems(const Geom& g) { return (size_t)4 * 2 * g.nb * 9 * 64; }

__device__ __forceinline__ size_t sp_index(const Geom& g, int par, int h, int k) {
  return ((size_t)(par * g.nb + (h >> 6)) * 12 + k) * 64 + (h & 63);
}
__device__ __forceinline__ size_t lk_index(const Geom& g, int mu, int par, int h, int k) {
  return ((size_t)((mu * 2 + par) * g.nb + (h >> 6)) * 9 + k) * 64 + (h & 63);
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
