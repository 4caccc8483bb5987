// Binary16 arithmetic shared by the FP16 Wilson operator and the FP16 network
// layers: packed (re, im) pairs, exact binary16 products summed in FP32
// (v_dot2_f32_f16), the SU(3) row-2 rebuild and link-times-vector products.
#pragma once
#include "common.h"

namespace qcd {

typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2v h2_of(__half2 x) { return __builtin_bit_cast(h2v, x); }
__device__ __forceinline__ h2v h_conjv(h2v x) {  // (re, -im)
  return __builtin_bit_cast(h2v, __builtin_bit_cast(uint32_t, x) ^ 0x80000000u);
}
__device__ __forceinline__ h2v h_swap(h2v x) { return h2v{x.y, x.x}; }     // (im, re)
__device__ __forceinline__ h2v h_muli(h2v x) { return h2v{-x.y, x.x}; }    // i x
__device__ __forceinline__ float hdot(h2v a, h2v b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }

// conj(x y - z w) = conj(x) conj(y) - conj(z) conj(w) in packed binary16
// arithmetic (one multiply and three fused multiply-adds on (re, im) pairs,
// each rounded to binary16, as the paper's FP16 arithmetic): the lane halves
// of x and z are broadcast and the swaps and signs of y and w fold into the
// instructions' operand selects and negations
__device__ __forceinline__ h2v h_rebuild(h2v x, h2v y, h2v z, h2v w) {
  h2v c = h2v{x.x, x.x} * h_conjv(y);                                  // (xr yr, -xr yi)
  c = __builtin_elementwise_fma(h2v{x.y, x.y}, -h_swap(y), c);          // conj(x y)
  c = __builtin_elementwise_fma(-h2v{z.x, z.x}, h_conjv(w), c);
  return __builtin_elementwise_fma(h2v{z.y, z.y}, h_swap(w), c);       // - conj(z w)
}
// row 2 = conj(row0 x row1), as su3_third_row
__device__ __forceinline__ void h_third_row(h2v (&u)[9]) {
  u[6] = h_rebuild(u[1], u[5], u[2], u[4]);
  u[7] = h_rebuild(u[2], u[3], u[0], u[5]);
  u[8] = h_rebuild(u[0], u[4], u[1], u[3]);
}

// The link in the form its products need: forward hops use (re, -im) and
// (im, re) of U_ab (Re and Im of U h), backward hops U_ab and i U_ab (Re and
// Im of U^dag h).
template <bool BWD> struct HLink { h2v p[9], q[9]; };
template <bool BWD> __device__ __forceinline__ void h_link_prep(const h2v (&u)[9], HLink<BWD>& L) {
#pragma unroll
  for (int k = 0; k < 9; k++) {
    if constexpr (!BWD) {
      L.p[k] = h_conjv(u[k]);
      L.q[k] = h_swap(u[k]);
    } else {
      L.p[k] = u[k];
      L.q[k] = h_muli(u[k]);
    }
  }
}
// w = U h (forward) or U^dag h (backward) in FP32
template <bool BWD>
__device__ __forceinline__ void h_mult(const HLink<BWD>& L, const h2v (&h)[3], cx<float> (&w)[3]) {
#pragma unroll
  for (int r = 0; r < 3; r++) {
    const int k0 = BWD ? r : 3 * r, dk = BWD ? 3 : 1;
    w[r].re = hdot(L.p[k0 + 2 * dk], h[2], hdot(L.p[k0 + dk], h[1], hdot(L.p[k0], h[0], 0.0f)));
    w[r].im = hdot(L.q[k0 + 2 * dk], h[2], hdot(L.q[k0 + dk], h[1], hdot(L.q[k0], h[0], 0.0f)));
  }
}

// w += U h (forward) or U^dag h (backward): the same products as h_mult with
// each chain starting from the accumulator instead of zero
template <bool BWD>
__device__ __forceinline__ void h_mult_acc(const HLink<BWD>& L, const h2v (&h)[3], cx<float> (&w)[3]) {
#pragma unroll
  for (int r = 0; r < 3; r++) {
    const int k0 = BWD ? r : 3 * r, dk = BWD ? 3 : 1;
    w[r].re = hdot(L.p[k0 + 2 * dk], h[2], hdot(L.p[k0 + dk], h[1], hdot(L.p[k0], h[0], w[r].re)));
    w[r].im = hdot(L.q[k0 + 2 * dk], h[2], hdot(L.q[k0 + dk], h[1], hdot(L.q[k0], h[0], w[r].im)));
  }
}

}  // namespace qcd
