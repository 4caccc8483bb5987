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

// conj(x y - z w) from binary16 entries: exact products, FP32 sums, one
// round-to-nearest-even conversion back to binary16
__device__ __forceinline__ h2v h_rebuild(h2v x, h2v y, h2v z, h2v w) {
  const h2v zn = -z;
  const float re = hdot(zn, h_conjv(w), hdot(x, h_conjv(y), 0.0f));
  const float im = hdot(zn, h_swap(w), hdot(x, h_swap(y), 0.0f));
  return h2v{(_Float16)re, (_Float16)(-im)};
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

}  // namespace qcd
