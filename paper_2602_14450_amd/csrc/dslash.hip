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
#include <type_traits>

#include "common.h"
#include "internal.h"
#include "half_ops.h"

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

// ---------------------------------------------------------------------------
// FP16 storage: the hop's arithmetic in native binary16 form.  The projection
// onto half-spinors is one packed binary16 add per complex component (one
// rounding, as the storage itself), and the SU(3) products use v_dot2_f32_f16:
// two binary16 products, exact, summed into an FP32 accumulator.  The
// reconstruction accumulates in FP32.  No spinor component is converted to
// FP32 before the link product.
// the projection of project<MU, MINUS> in binary16
template <int MU, bool MINUS>
__device__ __forceinline__ void project_h(const h2v (&f)[4][3], h2v (&h1)[3], h2v (&h2)[3]) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    if constexpr (MU == 0) {
      h1[c] = MINUS ? f[0][c] + h_muli(f[3][c]) : f[0][c] - h_muli(f[3][c]);
      h2[c] = MINUS ? f[1][c] + h_muli(f[2][c]) : f[1][c] - h_muli(f[2][c]);
    } else if constexpr (MU == 1) {
      h1[c] = MINUS ? f[0][c] + f[3][c] : f[0][c] - f[3][c];
      h2[c] = MINUS ? f[1][c] - f[2][c] : f[1][c] + f[2][c];
    } else if constexpr (MU == 2) {
      h1[c] = MINUS ? f[0][c] + h_muli(f[2][c]) : f[0][c] - h_muli(f[2][c]);
      h2[c] = MINUS ? f[1][c] - h_muli(f[3][c]) : f[1][c] + h_muli(f[3][c]);
    } else {
      h1[c] = MINUS ? f[2][c] + f[2][c] : f[0][c] + f[0][c];
      h2[c] = MINUS ? f[3][c] + f[3][c] : f[1][c] + f[1][c];
    }
  }
}

// Load the spinor granules a hop in direction MU needs: all of them, or for
// the t direction only those holding the spin pair its projector keeps.
template <int MU, bool MINUS, typename S, typename T>
__device__ __forceinline__ void load_spinor(const Geom& g, const S* __restrict__ in, int par, int h,
                                            cx<T> (&f)[4][3]) {
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C;
  const S* b = in + sp_block(g, par, h) + (h & 63) * C;
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++) {
    // components [jC, jC + C) hold spins (jC)/3 .. (jC + C - 1)/3
    const int s_lo = (j * C) / 3, s_hi = (j * C + C - 1) / 3;
    const bool need = (MU != 3) || (MINUS ? s_hi >= 2 : s_lo < 2);
    if (need) {
      const Gr v = *reinterpret_cast<const Gr*>(b + j * 64 * C);
#pragma unroll
      for (int c = 0; c < C; c++) {
        const int k = j * C + c;
        f[k / 3][k % 3] = Traits<S>::load(&v.s[c]);
      }
    }
  }
}

// Raw (still packed) data of one hop: the neighbour's spinor granules and
// the link granules (NE = 9 stored entries, or 6 with row 2 rebuilt).  Hops
// are numbered HOP = 2*mu + (0 forward, 1 backward).
template <typename S, int NE> struct HopRaw {
  typename Lay<S>::Gran sp[Lay<S>::G];
  typename Lay<S>::Gran lk[LkLay<S, NE>::F / Lay<S>::C];
  S tail[LkLay<S, NE>::TAIL > 0 ? LkLay<S, NE>::TAIL : 1];
};
template <typename S> struct alignas(2 * sizeof(S)) Pair { S s[2]; };

// Link loads.  A one-parity launch for one tile of right-hand sides reads
// every link of the lattice exactly once (each link joins an even and an odd
// site), so there the loads are marked non-temporal (LNT; 3% on the even-odd
// solve at 32^3 x 64).  A full launch reads each link twice, and the tiles of
// a multi-RHS launch read the same links again: both keep plain loads (the
// hint costs the full launch 8% and the 12-source batch 4%).
template <bool LNT, typename Gr> __device__ __forceinline__ Gr load_link_gran(const Gr* p) {
  if constexpr (LNT) return load_stream(p);
  else return *p;
}
template <bool LNT, typename S> __device__ __forceinline__ Pair<S> load_link_pair(const Pair<S>* p) {
  if constexpr (LNT && QCD_STREAM_HINTS) {
    static_assert(sizeof(Pair<S>) == 8, "a tail pair is 8 bytes");
    using V = unsigned int __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(Pair<S>, __builtin_nontemporal_load(reinterpret_cast<const V*>(p)));
  } else {
    return *p;
  }
}

// Spin pair a hop needs: the t-direction projectors keep spins (2,3) for
// (1 - g4) and (0,1) for (1 + g4); the others need all four.
template <int MU, bool MINUS, typename S> __device__ __forceinline__ constexpr bool gran_needed(int j) {
  constexpr int C = Lay<S>::C;
  return (MU != 3) || (MINUS ? (j * C + C - 1) / 3 >= 2 : (j * C) / 3 < 2);
}

template <int HOP, bool DAG, int NE, bool EO, bool LNT, typename S>
__device__ __forceinline__ void hop_load(const Geom& g, const S* __restrict__ in, const S* __restrict__ U, int par,
                                         int h, const Coord& c, HopRaw<S, NE>& d, int dep = 0) {
  constexpr int MU = HOP >> 1;
  constexpr bool BWD = HOP & 1;
  constexpr bool MINUS = BWD ? DAG : !DAG;  // forward hop of D uses (1 - gamma)
  constexpr int C = Lay<S>::C, F = LkLay<S, NE>::F, TAIL = LkLay<S, NE>::TAIL;
  using Gr = typename Lay<S>::Gran;
  int hn;
  if constexpr (MU == 0) {
    const int base = h - (c.x >> 1);
    const int xn = BWD ? ((c.x == 0) ? g.L[0] - 1 : c.x - 1) : ((c.x + 1 == g.L[0]) ? 0 : c.x + 1);
    hn = base + (xn >> 1);
  } else if constexpr (MU == 1) {
    hn = BWD ? ((c.y == 0) ? h + (g.L[1] - 1) * g.sy : h - g.sy) : ((c.y + 1 == g.L[1]) ? h - (g.L[1] - 1) * g.sy : h + g.sy);
  } else if constexpr (MU == 2) {
    hn = BWD ? ((c.z == 0) ? h + (g.L[2] - 1) * g.sz : h - g.sz) : ((c.z + 1 == g.L[2]) ? h - (g.L[2] - 1) * g.sz : h + g.sz);
  } else {
    hn = BWD ? ((c.t == 0) ? h + (g.L[3] - 1) * g.st : h - g.st) : ((c.t + 1 == g.L[3]) ? h - (g.L[3] - 1) * g.st : h + g.st);
  }
  hn += dep;  // dep is an opaque zero that orders these loads after an earlier hop
  const int npar = par ^ 1;
  // a one-parity input field holds only the neighbours' parity, indexed as parity 0
  const S* sb = in + sp_block(g, EO ? 0 : npar, hn) + (hn & 63) * C;
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++)
    if (gran_needed<MU, MINUS, S>(j)) d.sp[j] = *reinterpret_cast<const Gr*>(sb + j * 64 * C);
  // forward: U_mu(x) stored at x; backward: U_mu(x - mu) stored at the neighbour
  const int lp = BWD ? npar : par, lh = BWD ? hn : h + dep;
  const S* lb = U + lk_block<NE>(g, MU, lp, lh);
  const int lane = lh & 63;
#pragma unroll
  for (int j = 0; j < F / C; j++) d.lk[j] = load_link_gran<LNT>(reinterpret_cast<const Gr*>(lb + j * 64 * C + lane * C));
  if constexpr (NE == 9) {
#pragma unroll
    for (int k = F; k < 9; k++) d.tail[k - F] = lb[F * 64 + (k - F) * 64 + lane];
  } else if constexpr (TAIL == 2) {  // the two remaining entries of this lane, one 2-element load
    const Pair<S> v = load_link_pair<LNT>(reinterpret_cast<const Pair<S>*>(lb + F * 64 + lane * 2));
    d.tail[0] = v.s[0];
    d.tail[1] = v.s[1];
  } else {
    static_assert(TAIL == 0, "unsupported link layout");
  }
}

template <int HOP, bool DAG, int NE, typename S, typename T>
__device__ __forceinline__ T hop_compute(const HopRaw<S, NE>& d, cx<T> (&a)[4][3]) {
  constexpr int MU = HOP >> 1;
  constexpr bool BWD = HOP & 1;
  constexpr bool MINUS = BWD ? DAG : !DAG;
  constexpr int C = Lay<S>::C, F = LkLay<S, NE>::F;
  if constexpr (std::is_same<S, __half2>::value) {
    h2v f[4][3], u[9], h1[3], h2[3];
#pragma unroll
    for (int j = 0; j < Lay<S>::G; j++)
      if (gran_needed<MU, MINUS, S>(j)) {
#pragma unroll
        for (int cc = 0; cc < C; cc++) {
          const int k = j * C + cc;
          f[k / 3][k % 3] = h2_of(d.sp[j].s[cc]);
        }
      }
#pragma unroll
    for (int j = 0; j < F / C; j++)
#pragma unroll
      for (int cc = 0; cc < C; cc++) u[j * C + cc] = h2_of(d.lk[j].s[cc]);
#pragma unroll
    for (int k = F; k < NE; k++) u[k] = h2_of(d.tail[k - F]);
    if constexpr (NE == 6) h_third_row(u);
    project_h<MU, MINUS>(f, h1, h2);
    HLink<BWD> L;
    h_link_prep<BWD>(u, L);
    if constexpr (MU == 3) {
      // t hops: the projection keeps one spin half and the product adds to
      // that half alone, so its dot-product chains start from the accumulators
      constexpr int s0 = MINUS ? 2 : 0;
      h_mult_acc<BWD>(L, h1, a[s0]);
      h_mult_acc<BWD>(L, h2, a[s0 + 1]);
      return a[s0][0].re + a[s0 + 1][2].im;
    } else {
      cx<float> w1[3], w2[3];
      h_mult<BWD>(L, h1, w1);
      h_mult<BWD>(L, h2, w2);
      accumulate<MU, MINUS>(a, w1, w2);
      return w1[0].re + w2[2].im;
    }
  }
  cx<T> f[4][3], h1[3], h2[3], u[9], w1[3], w2[3];
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++)
    if (gran_needed<MU, MINUS, S>(j)) {
#pragma unroll
      for (int cc = 0; cc < C; cc++) {
        const int k = j * C + cc;
        f[k / 3][k % 3] = Traits<S>::load(&d.sp[j].s[cc]);
      }
    }
#pragma unroll
  for (int j = 0; j < F / C; j++)
#pragma unroll
    for (int cc = 0; cc < C; cc++) u[j * C + cc] = Traits<S>::load(&d.lk[j].s[cc]);
#pragma unroll
  for (int k = F; k < NE; k++) u[k] = Traits<S>::load(&d.tail[k - F]);
  if constexpr (NE == 6) su3_third_row(u);
  project<MU, MINUS>(f, h1, h2);
  if constexpr (!BWD) {  // U_mu(x) h
#pragma unroll
    for (int r = 0; r < 3; r++) {
      w1[r] = u[3 * r] * h1[0] + u[3 * r + 1] * h1[1] + u[3 * r + 2] * h1[2];
      w2[r] = u[3 * r] * h2[0] + u[3 * r + 1] * h2[1] + u[3 * r + 2] * h2[2];
    }
  } else {  // U_mu(x - mu)^dagger h
#pragma unroll
    for (int r = 0; r < 3; r++) {
      w1[r] = cmulc(u[r], h1[0]) + cmulc(u[3 + r], h1[1]) + cmulc(u[6 + r], h1[2]);
      w2[r] = cmulc(u[r], h2[0]) + cmulc(u[3 + r], h2[1]) + cmulc(u[6 + r], h2[2]);
    }
  }
  accumulate<MU, MINUS>(a, w1, w2);
  return w1[0].re + w2[2].im;  // a value that exists only once this hop is done
}

#define QCD_FENCE() __builtin_amdgcn_sched_barrier(0)

// Register barrier: the accumulators pass through empty asm statements as
// in/out operands, so every instruction producing them must be complete
// here and none of the hop's arithmetic can be sunk to the epilogue.
template <typename T> __device__ __forceinline__ void reg_barrier(cx<T> (&a)[4][3]) {
#pragma unroll
  for (int s = 0; s < 4; s++)
    asm volatile("" : "+v"(a[s][0].re), "+v"(a[s][0].im), "+v"(a[s][1].re), "+v"(a[s][1].im), "+v"(a[s][2].re),
                 "+v"(a[s][2].im));
}

// The eight hops as a software pipeline: before hop i is computed, the loads
// of hops i .. i+DEPTH are in flight.  The loads of hop i+DEPTH+1 are issued
// only after hop i is computed: their base pointers pass through an empty
// asm statement that takes hop i's product as an input, which the compiler
// must treat as a dependency.  This bounds the registers held by loaded data
// (otherwise all eight hops' loads are hoisted to the top and spilled).
struct PipeArgs {
  int par, h;
  Coord c;
};

template <int I, int DEPTH, bool DAG, int NE, bool EO, bool LNT, typename S, typename T>
__device__ __forceinline__ void hop_pipe(const Geom& g, const S* __restrict__ in, const S* __restrict__ U,
                                         const PipeArgs& pa, HopRaw<S, NE> (&buf)[DEPTH + 1], cx<T> (&a)[4][3]) {
  if constexpr (I < 8) {
    hop_compute<I, DAG, NE>(buf[I % (DEPTH + 1)], a);
    reg_barrier(a);
    if constexpr (I + DEPTH + 1 < 8) {
      int dep = 0;
      asm volatile("" : "+v"(dep) : "v"(a[0][0].re));
      hop_load<I + DEPTH + 1, DAG, NE, EO, LNT>(g, in, U, pa.par, pa.h, pa.c, buf[(I + DEPTH + 1) % (DEPTH + 1)], dep);
    }
    QCD_FENCE();
    hop_pipe<I + 1, DEPTH, DAG, NE, EO, LNT>(g, in, U, pa, buf, a);
  }
}

template <int I, int DEPTH, bool DAG, int NE, bool EO, bool LNT, typename S>
__device__ __forceinline__ void hop_prologue(const Geom& g, const S* __restrict__ in, const S* __restrict__ U,
                                             const PipeArgs& pa, HopRaw<S, NE> (&buf)[DEPTH + 1]) {
  if constexpr (I <= DEPTH) {
    hop_load<I, DAG, NE, EO, LNT>(g, in, U, pa.par, pa.h, pa.c, buf[I]);
    hop_prologue<I + 1, DEPTH, DAG, NE, EO, LNT>(g, in, U, pa, buf);
  }
}

template <int DEPTH, bool DAG, int NE, bool EO, bool LNT, typename S, typename T>
__device__ __forceinline__ void hop_all(const Geom& g, const S* __restrict__ in, const S* __restrict__ U, int par,
                                        int h, const Coord& c, cx<T> (&a)[4][3]) {
  HopRaw<S, NE> buf[DEPTH + 1];
  const PipeArgs pa{par, h, c};
  hop_prologue<0, DEPTH, DAG, NE, EO, LNT>(g, in, U, pa, buf);
  hop_pipe<0, DEPTH, DAG, NE, EO, LNT>(g, in, U, pa, buf, a);
}

// Whether a launch computes a right-hand side: mask 0 takes those whose inner
// solve is active, mask 1 those whose device-driven refinement step is due.
__device__ __forceinline__ bool scal_live(const Scalars& s, int mask) {
  return (mask ? s.outer_step : s.active) != 0;
}

// Thread -> (site, right-hand side).  A block of 256 threads is four waves:
// waves 0 and 1 take parity 0 and 1 of the first H/2 half indices of the
// block, waves 2 and 3 the next H/2, so the link a site reads as its forward
// link is read as the backward link of its neighbour by the same block.
// Within a wave, lane = s * T + r: 64/T sites times T right-hand sides, so
// the T lanes of one site request the same link granule in one instruction.
// With sched.mode 1 the blocks are ordered so that the eight XCDs (which
// receive consecutive workgroups in turn) each sweep their own slab of z in t
// order, all right-hand-side tiles of a site block back to back; this keeps
// t-neighbours and links inside that XCD's L2.  Mode 4 gives each XCD a slab
// of t instead, swept in z order (half the foreign faces when Lt = 2 Lz).
struct BlockPos { int h0, tile, sb; };
__device__ __forceinline__ BlockPos block_pos(const DslashSched& sc) {
  const int b = blockIdx.x;
  BlockPos p;
  if (sc.mode == 4) {
    // XCD xcd owns time slices [xcd*zc, (xcd+1)*zc) and sweeps them in z
    // order, all slices of one z plane (and all right-hand-side tiles) back
    // to back: z-neighbours stay in its L2 from the previous step, t-neighbours
    // are in the same step, and only the two slab faces in t are foreign
    const int xcd = b & 7, j = b >> 3;
    p.tile = j % sc.ntiles;
    const int js = j / sc.ntiles;
    const int per_z = sc.zc * sc.bp;
    const int z = js / per_z, rem = js - z * per_z;
    const int tl = rem / sc.bp, yb = rem - tl * sc.bp;
    p.sb = ((xcd * sc.zc + tl) * sc.Lz + z) * sc.bp + yb;
  } else if (sc.mode >= 1) {
    // XCD xcd owns z planes [xcd*zc, (xcd+1)*zc), swept as `sub` thinner
    // slabs one after the other, each in t order
    const int xcd = b & 7, j = b >> 3;
    p.tile = j % sc.ntiles;
    const int js = j / sc.ntiles;
    const int zs = sc.zc / sc.sub;            // z planes per sub-slab
    const int per_t = zs * sc.bp;
    const int per_sub = per_t * sc.Lt;
    const int sub = js / per_sub, r1 = js - sub * per_sub;
    const int t = r1 / per_t, rem = r1 - t * per_t;
    const int zl = rem / sc.bp, yb = rem - zl * sc.bp;
    p.sb = (t * sc.Lz + xcd * sc.zc + sub * zs + zl) * sc.bp + yb;
  } else {
    p.tile = b % sc.ntiles;
    p.sb = b / sc.ntiles;
  }
  p.h0 = p.sb * sc.H;
  return p;
}

// The centre term, the epilogue's sums and the store of one site's result
// (a: the site's hop sum; the reductions see the stored, rounded values).
template <typename S, int OP, int EPI, bool EO, int NV, typename T_>
__device__ __forceinline__ void site_finish(const Geom& g, S* __restrict__ out, const S* __restrict__ in,
                                            const S* __restrict__ cin, const S* __restrict__ aux, int fpar, int h,
                                            double kappa, int ftz, const cx<T_> (&a)[4][3], double (&red)[NV]) {
  constexpr bool TS = (EPI == kEpiTS || EPI == kEpiTSAux);
  const T_ k = (T_)kappa;
  cx<T_> o[12], ctr[12], ax[12];
  if constexpr (!(OP == kOpH || OP == kOpHdag)) {
    if constexpr (EO) load_site_stream(cin, g, fpar, h, ctr);  // read once
    else load_site(EO ? cin : in, g, fpar, h, ctr);  // the full form's centre is also neighbour data
  }
  if constexpr (EPI == kEpiResid || EPI == kEpiDotAux || EPI == kEpiTSAux) load_site_stream(aux, g, fpar, h, ax);
#pragma unroll
  for (int i = 0; i < 12; i++) {
    if constexpr (OP == kOpH || OP == kOpHdag) {
      o[i] = a[i / 3][i % 3];
    } else {
      o[i] = ctr[i] - k * a[i / 3][i % 3];
      if constexpr (EPI == kEpiResid) o[i] = ax[i] - o[i];
    }
  }
  // round to storage; the reductions see the stored values
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C;
  S* ob = out + sp_block(g, fpar, h) + (h & 63) * C;
  T_ acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
#pragma unroll
  for (int j = 0; j < Lay<S>::G; j++) {
    Gr v;
#pragma unroll
    for (int cc = 0; cc < C; cc++) {
      const int i = j * C + cc;
      v.s[cc] = Traits<S>::pack(o[i], ftz);
      if constexpr (EPI != kEpiNone) {
        const cx<T_> os = Traits<S>::load(&v.s[cc]);
        if constexpr (EPI == kEpiDotAux) {  // (aux, out) = sum conj(aux) out
          acc0 += ax[i].re * os.re + ax[i].im * os.im;
          acc1 += ax[i].re * os.im - ax[i].im * os.re;
        } else if constexpr (TS) {  // (t, s) with t = out, s = in (TS) or aux (TSAux); |t|^2, |s|^2
          const cx<T_> sv = (EPI == kEpiTSAux) ? ax[i] : ctr[i];
          acc0 += os.re * sv.re + os.im * sv.im;
          acc1 += os.re * sv.im - os.im * sv.re;
          acc2 += norm2(os);
          acc3 += norm2(sv);
        } else if constexpr (EPI == kEpiRecon) {  // cin - (out - |kappa| H in), as a separate residual launch forms it
          const cx<T_> dv = os - (-k) * a[i / 3][i % 3];
          acc0 += norm2(ctr[i] - dv);
        } else {
          acc0 += norm2(os);
        }
      }
    }
    store_stream(reinterpret_cast<Gr*>(ob + j * 64 * C), v);
  }
  if constexpr (EPI == kEpiDotAux) { red[0] = acc0; red[1] = acc1; }
  if constexpr (TS) { red[0] = acc0; red[1] = acc1; red[2] = acc2; red[3] = acc3; }
  if constexpr (EPI == kEpiResid || EPI == kEpiRecon) { red[0] = acc0; }
}

// out = D in, H in, D^dag in, or b - D in, with optional reduction epilogues,
// for T right-hand sides per wave (vectors of right-hand side r start at
// r * vstride elements).  With EO the output covers parity tpar only and every
// vector is a one-parity field: the hops read `in` (the other parity) and D's
// centre term comes from `cin` (parity tpar), so out = cin - kappa H in
// (kappa = kappa^2 gives the Schur complement's second half, kappa < 0 the
// right-hand side and the reconstruction of the even-odd solve).
template <typename S, int OP, int EPI, int DEPTH, int OCC, int T, int NE, bool EO, bool LNT>
__global__ __launch_bounds__(256, OCC) void k_dslash(Geom g, DslashSched sched, S* __restrict__ out,
                                                     const S* __restrict__ in, const S* __restrict__ U, double kappa,
                                                     const S* __restrict__ aux, double* __restrict__ partials,
                                                     const Scalars* __restrict__ scal, int ftz,
                                                     const S* __restrict__ cin, int tpar, int mask) {
  using T_ = typename Traits<S>::T;
  const BlockPos bp = block_pos(sched);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int r = lane % T;
  const int rhs = bp.tile * T + r;
  if (scal) {  // skip blocks whose right-hand sides have all stopped
    bool any = false;
#pragma unroll
    for (int i = 0; i < T; i++) any |= scal_live(scal[bp.tile * T + i], mask);
    if (!any) return;
  }
  const bool live = !scal || scal_live(scal[rhs], mask);
  const int par = EO ? tpar : (wid & 1);
  const int h = EO ? bp.h0 + wid * (64 / T) + lane / T : bp.h0 + (wid >> 1) * (64 / T) + lane / T;
  const int fpar = EO ? 0 : par;  // parity index of this site in its own fields
  const size_t vo = (size_t)rhs * (EO ? (size_t)g.nb * 768 : spinor_elems(g));
  in += vo;
  out += vo;
  if (aux) aux += vo;
  if (EO && cin) cin += vo;
  constexpr bool DAG = (OP == kOpDdag || OP == kOpHdag);
  constexpr bool TS = (EPI == kEpiTS || EPI == kEpiTSAux);
  constexpr int NV = (EPI == kEpiNone) ? 1 : (EPI == kEpiDotAux ? 2 : (TS ? 4 : 1));
  static_assert(EPI != kEpiRecon || (EO && OP == kOpD), "the reconstruction epilogue is a one-parity D form");
  double red[NV];
#pragma unroll
  for (int i = 0; i < NV; i++) red[i] = 0.0;
  if (h < g.Vh && live) {
    const Coord c = decode(g, par, h);
    cx<T_> a[4][3];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int cc = 0; cc < 3; cc++) a[s][cc] = cx<T_>(0, 0);
    hop_all<DEPTH, DAG, NE, EO, LNT>(g, in, U, par, h, c, a);
    site_finish<S, OP, EPI, EO, NV>(g, out, in, cin, aux, fpar, h, kappa, ftz, a, red);
  }
  if constexpr (EPI != kEpiNone) block_reduce_store_T<NV, T>(red, partials, bp.tile * T, sched.nsb, bp.sb);
}

// ---------------------------------------------------------------------------
// The operator with the x and y neighbours staged in LDS (full lattice, one
// right-hand side per thread, no reduction epilogue; launch variant 6).  A
// block covers R = H / (Lx/2) whole x rows of both parities at one (z, t)
// (H = 128 half sites per parity); it stages its own sites and the rows
// y0 - 1 and y0 + R of both parities once, as 16-byte granules laid out
// [parity][granule][row][x/2] so that a wave reading one granule reads
// consecutive LDS words, and the x and y hops and the centre term take their
// spinors from there.  Links and the z and t neighbours come from global memory.
template <int MU, bool BWD> __device__ __forceinline__ int hop_neighbour(const Geom& g, int h, const Coord& c);

constexpr int kLdsMaxLxh = 64;                       // Lx <= 128
constexpr int kLdsEntries = 128 + 2 * kLdsMaxLxh;    // (R + 2) * (Lx/2) half sites at most per parity

template <typename S> struct LdsTile {
  const typename Lay<S>::Gran* t;  // LDS granules [parity][granule][row][x/2]
  int rows, lxh;
  __device__ __forceinline__ const typename Lay<S>::Gran& at(int par, int j, int row, int xh) const {
    return t[((par * Lay<S>::G + j) * rows + row) * lxh + xh];
  }
};

// The hop's link granules (as hop_load): U_mu(x) at (par, h) forward, U_mu(x - mu) at (par ^ 1, hn) backward.
template <int HOP, int NE, bool LNT, typename S>
__device__ __forceinline__ void hop_load_link(const Geom& g, const S* __restrict__ U, int par, int h, int hn,
                                              HopRaw<S, NE>& d) {
  constexpr int MU = HOP >> 1;
  constexpr bool BWD = HOP & 1;
  constexpr int C = Lay<S>::C, F = LkLay<S, NE>::F, TAIL = LkLay<S, NE>::TAIL;
  using Gr = typename Lay<S>::Gran;
  const int lp = BWD ? (par ^ 1) : par, lh = BWD ? hn : h;
  const S* lb = U + lk_block<NE>(g, MU, lp, lh);
  const int lane = lh & 63;
#pragma unroll
  for (int j = 0; j < F / C; j++) d.lk[j] = load_link_gran<LNT>(reinterpret_cast<const Gr*>(lb + j * 64 * C + lane * C));
  if constexpr (NE == 9) {
#pragma unroll
    for (int k = F; k < 9; k++) d.tail[k - F] = lb[F * 64 + (k - F) * 64 + lane];
  } else if constexpr (TAIL == 2) {
    const Pair<S> v = load_link_pair<LNT>(reinterpret_cast<const Pair<S>*>(lb + F * 64 + lane * 2));
    d.tail[0] = v.s[0];
    d.tail[1] = v.s[1];
  }
}

// hop_load with the x and y neighbours' spinors from the LDS tile (row and xh
// locate this site in it; rows are offset by the halo row).  The one-parity
// form's tile holds the input field's single parity.
template <int HOP, bool DAG, int NE, bool EO, bool LNT, typename S>
__device__ __forceinline__ void hop_load_lds(const Geom& g, const S* __restrict__ in, const S* __restrict__ U,
                                             int par, int h, const Coord& c, int row, int xh, const LdsTile<S>& L,
                                             HopRaw<S, NE>& d, int dep = 0) {
  constexpr int MU = HOP >> 1;
  constexpr bool BWD = HOP & 1;
  constexpr bool MINUS = BWD ? DAG : !DAG;
  if constexpr (MU >= 2) {
    hop_load<HOP, DAG, NE, EO, LNT>(g, in, U, par, h, c, d, dep);
  } else {
    const int hn = hop_neighbour<MU, BWD>(g, h, c) + dep;
    int rn = row + dep, xn = xh;
    if constexpr (MU == 0) {
      const int xx = BWD ? ((c.x == 0) ? g.L[0] - 1 : c.x - 1) : ((c.x + 1 == g.L[0]) ? 0 : c.x + 1);
      xn = xx >> 1;
    } else {
      rn += BWD ? -1 : 1;
    }
#pragma unroll
    for (int j = 0; j < Lay<S>::G; j++)
      if (gran_needed<MU, MINUS, S>(j)) d.sp[j] = L.at(EO ? 0 : par ^ 1, j, rn, xn);
    hop_load_link<HOP, NE, LNT>(g, U, par, h + dep, hn, d);
  }
}

template <int I, int DEPTH, bool DAG, int NE, bool EO, bool LNT, typename S, typename T>
__device__ __forceinline__ void hop_pipe_lds(const Geom& g, const S* __restrict__ in, const S* __restrict__ U,
                                             const PipeArgs& pa, int row, int xh, const LdsTile<S>& L,
                                             HopRaw<S, NE> (&buf)[DEPTH + 1], cx<T> (&a)[4][3]) {
  if constexpr (I < 8) {
    hop_compute<I, DAG, NE>(buf[I % (DEPTH + 1)], a);
    reg_barrier(a);
    if constexpr (I + DEPTH + 1 < 8) {
      int dep = 0;
      asm volatile("" : "+v"(dep) : "v"(a[0][0].re));
      hop_load_lds<I + DEPTH + 1, DAG, NE, EO, LNT>(g, in, U, pa.par, pa.h, pa.c, row, xh, L,
                                           buf[(I + DEPTH + 1) % (DEPTH + 1)], dep);
    }
    QCD_FENCE();
    hop_pipe_lds<I + 1, DEPTH, DAG, NE, EO, LNT>(g, in, U, pa, row, xh, L, buf, a);
  }
}

template <int I, int DEPTH, bool DAG, int NE, bool EO, bool LNT, typename S>
__device__ __forceinline__ void hop_prologue_lds(const Geom& g, const S* __restrict__ in, const S* __restrict__ U,
                                                 const PipeArgs& pa, int row, int xh, const LdsTile<S>& L,
                                                 HopRaw<S, NE> (&buf)[DEPTH + 1]) {
  if constexpr (I <= DEPTH) {
    hop_load_lds<I, DAG, NE, EO, LNT>(g, in, U, pa.par, pa.h, pa.c, row, xh, L, buf[I]);
    hop_prologue_lds<I + 1, DEPTH, DAG, NE, EO, LNT>(g, in, U, pa, row, xh, L, buf);
  }
}

// Whether the LDS form applies: blocks of H = 128 half sites cover whole x rows of one (z, t) plane.
inline bool lds_form_applies(const Geom& g) {
  const int R = 128 / g.Lxh;
  return g.Lxh <= kLdsMaxLxh && 128 % g.Lxh == 0 && g.L[1] % R == 0;
}

template <typename S, int OP, int DEPTH, int NE>
__global__ __launch_bounds__(256, 2) void k_dslash_lds(Geom g, DslashSched sched, S* __restrict__ out,
                                                       const S* __restrict__ in, const S* __restrict__ U,
                                                       double kappa, int ftz) {
  using T_ = typename Traits<S>::T;
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C, G = Lay<S>::G;
  constexpr bool DAG = (OP == kOpDdag || OP == kOpHdag);
  __shared__ Gr tile[2 * G * kLdsEntries];
  const BlockPos bp = block_pos(sched);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int lxh = g.Lxh, R = 128 / lxh, rows = R + 2;
  const LdsTile<S> L{tile, rows, lxh};
  const int par = wid & 1;
  const int j = (wid >> 1) * 64 + lane;  // half site within the block
  const int h = bp.h0 + j;
  const int row = j / lxh + 1, xh = j - (j / lxh) * lxh;
  // the block's rows: plane base and the y of its first row
  const int y0 = (bp.h0 / lxh) % g.L[1];
  const int pbase = bp.h0 - y0 * lxh;
  // stage the block's own sites
  if (h < g.Vh) {
    const S* b = in + sp_block(g, par, h) + (h & 63) * C;
#pragma unroll
    for (int k = 0; k < G; k++) tile[((par * G + k) * rows + row) * lxh + xh] = *reinterpret_cast<const Gr*>(b + k * 64 * C);
  }
  // and the rows above and below, both parities
  for (int k = tid; k < 2 * 2 * lxh * G; k += 256) {
    const int jg = k % G, r1 = k / G;
    const int xs = r1 % lxh, r2 = r1 / lxh;
    const int which = r2 & 1, hp = r2 >> 1;
    const int yy = which ? (y0 + R) % g.L[1] : (y0 + g.L[1] - 1) % g.L[1];
    const int hh = pbase + yy * lxh + xs;
    tile[((hp * G + jg) * rows + (which ? R + 1 : 0)) * lxh + xs] =
        *reinterpret_cast<const Gr*>(in + sp_block(g, hp, hh) + (hh & 63) * C + jg * 64 * C);
  }
  __syncthreads();
  if (h >= g.Vh) return;
  const Coord c = decode(g, par, h);
  cx<T_> a[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; sp++)
#pragma unroll
    for (int cc = 0; cc < 3; cc++) a[sp][cc] = cx<T_>(0, 0);
  {
    HopRaw<S, NE> buf[DEPTH + 1];
    const PipeArgs pa{par, h, c};
    hop_prologue_lds<0, DEPTH, DAG, NE, false, false>(g, in, U, pa, row, xh, L, buf);
    hop_pipe_lds<0, DEPTH, DAG, NE, false, false>(g, in, U, pa, row, xh, L, buf, a);
  }
  const T_ k = (T_)kappa;
  S* ob = out + sp_block(g, par, h) + (h & 63) * C;
#pragma unroll
  for (int jj = 0; jj < G; jj++) {
    const Gr cv = L.at(par, jj, row, xh);
    Gr v;
#pragma unroll
    for (int cc = 0; cc < C; cc++) {
      const int i = jj * C + cc;
      cx<T_> o = a[i / 3][i % 3];
      if constexpr (!(OP == kOpH || OP == kOpHdag)) {
        const cx<T_> ctr = Traits<S>::load(&cv.s[cc]);
        o = ctr - k * o;
      }
      v.s[cc] = Traits<S>::pack(o, ftz);
    }
    store_stream(reinterpret_cast<Gr*>(ob + jj * 64 * C), v);
  }
}

// The one-parity operator of the even-odd form with the x and y neighbours in
// LDS (one right-hand side per launch tile, every epilogue; variant 6).  A
// block covers H = 256 half sites of the output parity, R = H / (Lx/2) whole
// x rows at one (z, t); the input field (the other parity) is staged for
// those rows and the rows y0 - 1 and y0 + R.  The centre term, the auxiliary
// vectors, the links and the z and t neighbours come from global memory, as
// in k_dslash.
// Rows of at most 64 half sites (32 for FP64 spinors, which keeps the tile
// within 64 KB: 320 x 192 B).
template <typename S> struct LdsEo {
  static constexpr int kMaxLxh = Lay<S>::G > 6 ? 32 : 64;
  static constexpr int kEntries = 256 + 2 * kMaxLxh;
};

template <typename S> inline bool lds_eo_form_applies(const Geom& g) {
  const int R = 256 / g.Lxh;
  return g.Lxh <= LdsEo<S>::kMaxLxh && 256 % g.Lxh == 0 && g.L[1] % R == 0;
}

template <typename S, int OP, int EPI, int DEPTH, int NE>
__global__ __launch_bounds__(256, 2) void k_dslash_lds_eo(Geom g, DslashSched sched, S* __restrict__ out,
                                                          const S* __restrict__ in, const S* __restrict__ U,
                                                          double kappa, const S* __restrict__ aux,
                                                          double* __restrict__ partials,
                                                          const Scalars* __restrict__ scal, int ftz,
                                                          const S* __restrict__ cin, int tpar, int mask) {
  using T_ = typename Traits<S>::T;
  using Gr = typename Lay<S>::Gran;
  constexpr int C = Lay<S>::C, G = Lay<S>::G;
  constexpr bool DAG = (OP == kOpDdag || OP == kOpHdag);
  constexpr bool TS = (EPI == kEpiTS || EPI == kEpiTSAux);
  constexpr int NV = (EPI == kEpiNone) ? 1 : (EPI == kEpiDotAux ? 2 : (TS ? 4 : 1));
  __shared__ Gr tile[G * LdsEo<S>::kEntries];
  const BlockPos bp = block_pos(sched);
  const int rhs = bp.tile;
  if (scal && !scal_live(scal[rhs], mask)) return;  // the whole block belongs to one right-hand side
  const int tid = threadIdx.x;
  const int h = bp.h0 + tid;
  const size_t vo = (size_t)rhs * (size_t)g.nb * 768;
  in += vo;
  out += vo;
  if (aux) aux += vo;
  if (cin) cin += vo;
  const int lxh = g.Lxh, R = 256 / lxh, rows = R + 2;
  const LdsTile<S> L{tile, rows, lxh};
  const int row = tid / lxh + 1, xh = tid - (tid / lxh) * lxh;
  const int y0 = (bp.h0 / lxh) % g.L[1];
  const int pbase = bp.h0 - y0 * lxh;
  {  // the input field on the block's rows (same half index, the other parity) ...
    const S* b = in + sp_block(g, 0, h) + (h & 63) * C;
#pragma unroll
    for (int k = 0; k < G; k++) tile[(k * rows + row) * lxh + xh] = *reinterpret_cast<const Gr*>(b + k * 64 * C);
  }
  // ... and on the rows above and below
  for (int k = tid; k < 2 * lxh * G; k += 256) {
    const int jg = k % G, r1 = k / G;
    const int xs = r1 % lxh, which = r1 / lxh;
    const int yy = which ? (y0 + R) % g.L[1] : (y0 + g.L[1] - 1) % g.L[1];
    const int hh = pbase + yy * lxh + xs;
    tile[(jg * rows + (which ? R + 1 : 0)) * lxh + xs] =
        *reinterpret_cast<const Gr*>(in + sp_block(g, 0, hh) + (hh & 63) * C + jg * 64 * C);
  }
  __syncthreads();
  double red[NV];
#pragma unroll
  for (int i = 0; i < NV; i++) red[i] = 0.0;
  {
    const Coord c = decode(g, tpar, h);
    cx<T_> a[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; sp++)
#pragma unroll
      for (int cc = 0; cc < 3; cc++) a[sp][cc] = cx<T_>(0, 0);
    {
      HopRaw<S, NE> buf[DEPTH + 1];
      const PipeArgs pa{tpar, h, c};
      hop_prologue_lds<0, DEPTH, DAG, NE, true, true>(g, in, U, pa, row, xh, L, buf);
      hop_pipe_lds<0, DEPTH, DAG, NE, true, true>(g, in, U, pa, row, xh, L, buf, a);
    }
    site_finish<S, OP, EPI, true, NV>(g, out, in, cin, aux, 0, h, kappa, ftz, a, red);
  }
  if constexpr (EPI != kEpiNone) block_reduce_store_T<NV, 1>(red, partials, rhs, sched.nsb, bp.sb);
}

// ---------------------------------------------------------------------------
// Several right-hand sides per thread: the thread of a site applies the link
// it loaded (and rebuilt) once to R right-hand sides, so the link conversion,
// the row-2 rebuild and the neighbour addressing are paid once per site
// rather than once per site and right-hand side (the FP16 operator is bound by
// instruction issue, not bytes).

template <typename S, int NE, int R> struct HopRawR {
  typename Lay<S>::Gran sp[R][Lay<S>::G];
  typename Lay<S>::Gran lk[LkLay<S, NE>::F / Lay<S>::C];
  S tail[LkLay<S, NE>::TAIL > 0 ? LkLay<S, NE>::TAIL : 1];
};

template <int MU, bool BWD>
__device__ __forceinline__ int hop_neighbour(const Geom& g, int h, const Coord& c) {
  if constexpr (MU == 0) {
    const int base = h - (c.x >> 1);
    const int xn = BWD ? ((c.x == 0) ? g.L[0] - 1 : c.x - 1) : ((c.x + 1 == g.L[0]) ? 0 : c.x + 1);
    return base + (xn >> 1);
  } else if constexpr (MU == 1) {
    return BWD ? ((c.y == 0) ? h + (g.L[1] - 1) * g.sy : h - g.sy) : ((c.y + 1 == g.L[1]) ? h - (g.L[1] - 1) * g.sy : h + g.sy);
  } else if constexpr (MU == 2) {
    return BWD ? ((c.z == 0) ? h + (g.L[2] - 1) * g.sz : h - g.sz) : ((c.z + 1 == g.L[2]) ? h - (g.L[2] - 1) * g.sz : h + g.sz);
  } else {
    return BWD ? ((c.t == 0) ? h + (g.L[3] - 1) * g.st : h - g.st) : ((c.t + 1 == g.L[3]) ? h - (g.L[3] - 1) * g.st : h + g.st);
  }
}

template <int HOP, bool DAG, int NE, int R, bool EO, typename S>
__device__ __forceinline__ void hop_load_r(const Geom& g, const S* __restrict__ in, size_t vstride,
                                           const S* __restrict__ U, int par, int h, const Coord& c,
                                           HopRawR<S, NE, R>& d, int dep = 0) {
  constexpr int MU = HOP >> 1;
  constexpr bool BWD = HOP & 1;
  constexpr bool MINUS = BWD ? DAG : !DAG;
  constexpr int C = Lay<S>::C, F = LkLay<S, NE>::F, TAIL = LkLay<S, NE>::TAIL;
  using Gr = typename Lay<S>::Gran;
  const int hn = hop_neighbour<MU, BWD>(g, h, c) + dep;
  const int npar = par ^ 1;
  const S* sb = in + sp_block(g, EO ? 0 : npar, hn) + (hn & 63) * C;
#pragma unroll
  for (int r = 0; r < R; r++)
#pragma unroll
    for (int j = 0; j < Lay<S>::G; j++)
      if (gran_needed<MU, MINUS, S>(j)) d.sp[r][j] = *reinterpret_cast<const Gr*>(sb + r * vstride + j * 64 * C);
  const int lp = BWD ? npar : par, lh = BWD ? hn : h + dep;
  const S* lb = U + lk_block<NE>(g, MU, lp, lh);
  const int lane = lh & 63;
#pragma unroll
  for (int j = 0; j < F / C; j++) d.lk[j] = load_link_gran<false>(reinterpret_cast<const Gr*>(lb + j * 64 * C + lane * C));
  if constexpr (NE == 9) {
#pragma unroll
    for (int k = F; k < 9; k++) d.tail[k - F] = lb[F * 64 + (k - F) * 64 + lane];
  } else if constexpr (TAIL == 2) {
    const Pair<S> v = load_link_pair<false>(reinterpret_cast<const Pair<S>*>(lb + F * 64 + lane * 2));
    d.tail[0] = v.s[0];
    d.tail[1] = v.s[1];
  }
}

template <int HOP, bool DAG, int NE, int R, typename S, typename T>
__device__ __forceinline__ void hop_compute_r(const HopRawR<S, NE, R>& d, cx<T> (&a)[R][4][3]) {
  constexpr int MU = HOP >> 1;
  constexpr bool BWD = HOP & 1;
  constexpr bool MINUS = BWD ? DAG : !DAG;
  constexpr int C = Lay<S>::C, F = LkLay<S, NE>::F;
  if constexpr (std::is_same<S, __half2>::value) {
    h2v u[9];
#pragma unroll
    for (int j = 0; j < F / C; j++)
#pragma unroll
      for (int cc = 0; cc < C; cc++) u[j * C + cc] = h2_of(d.lk[j].s[cc]);
#pragma unroll
    for (int k = F; k < NE; k++) u[k] = h2_of(d.tail[k - F]);
    if constexpr (NE == 6) h_third_row(u);
    HLink<BWD> L;
    h_link_prep<BWD>(u, L);
#pragma unroll
    for (int r = 0; r < R; r++) {
      h2v f[4][3], h1[3], h2[3];
#pragma unroll
      for (int j = 0; j < Lay<S>::G; j++)
        if (gran_needed<MU, MINUS, S>(j)) {
#pragma unroll
          for (int cc = 0; cc < C; cc++) {
            const int k = j * C + cc;
            f[k / 3][k % 3] = h2_of(d.sp[r][j].s[cc]);
          }
        }
      project_h<MU, MINUS>(f, h1, h2);
      if constexpr (MU == 3) {  // as in hop_compute: chains start from the accumulators
        constexpr int s0 = MINUS ? 2 : 0;
        h_mult_acc<BWD>(L, h1, a[r][s0]);
        h_mult_acc<BWD>(L, h2, a[r][s0 + 1]);
      } else {
        cx<float> w1[3], w2[3];
        h_mult<BWD>(L, h1, w1);
        h_mult<BWD>(L, h2, w2);
        accumulate<MU, MINUS>(a[r], w1, w2);
      }
    }
    return;
  }
  cx<T> u[9];
#pragma unroll
  for (int j = 0; j < F / C; j++)
#pragma unroll
    for (int cc = 0; cc < C; cc++) u[j * C + cc] = Traits<S>::load(&d.lk[j].s[cc]);
#pragma unroll
  for (int k = F; k < NE; k++) u[k] = Traits<S>::load(&d.tail[k - F]);
  if constexpr (NE == 6) su3_third_row(u);
#pragma unroll
  for (int r = 0; r < R; r++) {
    cx<T> f[4][3], h1[3], h2[3], w1[3], w2[3];
#pragma unroll
    for (int j = 0; j < Lay<S>::G; j++)
      if (gran_needed<MU, MINUS, S>(j)) {
#pragma unroll
        for (int cc = 0; cc < C; cc++) {
          const int k = j * C + cc;
          f[k / 3][k % 3] = Traits<S>::load(&d.sp[r][j].s[cc]);
        }
      }
    project<MU, MINUS>(f, h1, h2);
    if constexpr (!BWD) {
#pragma unroll
      for (int q = 0; q < 3; q++) {
        w1[q] = u[3 * q] * h1[0] + u[3 * q + 1] * h1[1] + u[3 * q + 2] * h1[2];
        w2[q] = u[3 * q] * h2[0] + u[3 * q + 1] * h2[1] + u[3 * q + 2] * h2[2];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 3; q++) {
        w1[q] = cmulc(u[q], h1[0]) + cmulc(u[3 + q], h1[1]) + cmulc(u[6 + q], h1[2]);
        w2[q] = cmulc(u[q], h2[0]) + cmulc(u[3 + q], h2[1]) + cmulc(u[6 + q], h2[2]);
      }
    }
    accumulate<MU, MINUS>(a[r], w1, w2);
  }
}

template <int R, typename T> __device__ __forceinline__ void reg_barrier_r(cx<T> (&a)[R][4][3]) {
#pragma unroll
  for (int r = 0; r < R; r++) reg_barrier(a[r]);
}

// The eight hops one after the other; the loads of hop i+1 are issued after
// hop i is computed (dependency through an empty asm statement).
template <int I, bool DAG, int NE, int R, bool EO, typename S, typename T>
__device__ __forceinline__ void hop_seq_r(const Geom& g, const S* __restrict__ in, size_t vstride,
                                          const S* __restrict__ U, int par, int h, const Coord& c,
                                          cx<T> (&a)[R][4][3], int dep) {
  if constexpr (I < 8) {
    HopRawR<S, NE, R> d;
    hop_load_r<I, DAG, NE, R, EO>(g, in, vstride, U, par, h, c, d, dep);
    hop_compute_r<I, DAG, NE, R>(d, a);
    reg_barrier_r<R>(a);
    int dep2 = 0;
    asm volatile("" : "+v"(dep2) : "v"(a[0][0][0].re));
    QCD_FENCE();
    hop_seq_r<I + 1, DAG, NE, R, EO>(g, in, vstride, U, par, h, c, a, dep2);
  }
}

// Per-right-hand-side block reduction for R right-hand sides per thread:
// value i of right-hand side r0 + r goes to partials[((r0 + r) * rstride + row) * NV + i].
template <int NV, int R>
__device__ __forceinline__ void block_reduce_store_R(double (&v)[R][NV], double* partials, int r0, int rstride,
                                                     int row) {
  __shared__ double red[R * NV][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < R; r++)
#pragma unroll
    for (int i = 0; i < NV; i++) {
      double a = v[r][i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
      if (lane == 0) red[r * NV + i][wid] = a;
    }
  __syncthreads();
  if ((int)threadIdx.x < R * NV) {
    const int r = threadIdx.x / NV, i = threadIdx.x % NV;
    const double s = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) + red[threadIdx.x][3];
    partials[((size_t)(r0 + r) * rstride + row) * NV + i] = s;
  }
}

// EO as in k_dslash: one parity tpar of one-parity fields, centre term from cin.
template <typename S, int OP, int EPI, int R, int NE, bool EO>
__global__ __launch_bounds__(256, 2) void k_dslash_mr(Geom g, DslashSched sched, S* __restrict__ out,
                                                      const S* __restrict__ in, const S* __restrict__ U, double kappa,
                                                      const S* __restrict__ aux, double* __restrict__ partials,
                                                      const Scalars* __restrict__ scal, int ftz,
                                                      const S* __restrict__ cin, int tpar, int mask) {
  using T_ = typename Traits<S>::T;
  const BlockPos bp = block_pos(sched);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r0 = bp.tile * R;
  bool live[R];
  bool any = false;
#pragma unroll
  for (int r = 0; r < R; r++) {
    live[r] = !scal || scal_live(scal[r0 + r], mask);
    any |= live[r];
  }
  if (!any) return;  // uniform over the block
  const int par = EO ? tpar : (wid & 1);
  const int h = EO ? bp.h0 + wid * 64 + lane : bp.h0 + (wid >> 1) * 64 + lane;
  const int fpar = EO ? 0 : par;
  const size_t vs = EO ? (size_t)g.nb * 768 : spinor_elems(g);
  const size_t vo = (size_t)r0 * vs;
  constexpr bool DAG = (OP == kOpDdag || OP == kOpHdag);
  constexpr bool TS = (EPI == kEpiTS || EPI == kEpiTSAux);
  constexpr int NV = (EPI == kEpiNone) ? 1 : (EPI == kEpiDotAux ? 2 : (TS ? 4 : 1));
  double red[R][NV];
#pragma unroll
  for (int r = 0; r < R; r++)
#pragma unroll
    for (int i = 0; i < NV; i++) red[r][i] = 0.0;
  if (h < g.Vh) {
    const Coord c = decode(g, par, h);
    cx<T_> a[R][4][3];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
      for (int sp = 0; sp < 4; sp++)
#pragma unroll
        for (int cc = 0; cc < 3; cc++) a[r][sp][cc] = cx<T_>(0, 0);
    hop_seq_r<0, DAG, NE, R, EO>(g, in + vo, vs, U, par, h, c, a, 0);
    const T_ k = (T_)kappa;
    using Gr = typename Lay<S>::Gran;
    constexpr int C = Lay<S>::C;
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (!live[r]) continue;
      const S* inr = (EO ? cin : in) + vo + r * vs;
      const S* axr = aux ? aux + vo + r * vs : nullptr;
      cx<T_> o[12], ctr[12], ax[12];
      if constexpr (!(OP == kOpH || OP == kOpHdag)) {
        if constexpr (EO) load_site_stream(inr, g, fpar, h, ctr);
        else load_site(inr, g, fpar, h, ctr);
      }
      if constexpr (EPI == kEpiResid || EPI == kEpiDotAux || EPI == kEpiTSAux) load_site_stream(axr, g, fpar, h, ax);
#pragma unroll
      for (int i = 0; i < 12; i++) {
        if constexpr (OP == kOpH || OP == kOpHdag) {
          o[i] = a[r][i / 3][i % 3];
        } else {
          o[i] = ctr[i] - k * a[r][i / 3][i % 3];
          if constexpr (EPI == kEpiResid) o[i] = ax[i] - o[i];
        }
      }
      S* ob = out + vo + r * vs + sp_block(g, fpar, h) + (h & 63) * C;
      T_ acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
#pragma unroll
      for (int j = 0; j < Lay<S>::G; j++) {
        Gr v;
#pragma unroll
        for (int cc = 0; cc < C; cc++) {
          const int i = j * C + cc;
          v.s[cc] = Traits<S>::pack(o[i], ftz);
          if constexpr (EPI != kEpiNone) {
            const cx<T_> os = Traits<S>::load(&v.s[cc]);
            if constexpr (EPI == kEpiDotAux) {
              acc0 += ax[i].re * os.re + ax[i].im * os.im;
              acc1 += ax[i].re * os.im - ax[i].im * os.re;
            } else if constexpr (TS) {
              const cx<T_> sv = (EPI == kEpiTSAux) ? ax[i] : ctr[i];
              acc0 += os.re * sv.re + os.im * sv.im;
              acc1 += os.re * sv.im - os.im * sv.re;
              acc2 += norm2(os);
              acc3 += norm2(sv);
            } else {
              acc0 += norm2(os);
            }
          }
        }
        store_stream(reinterpret_cast<Gr*>(ob + j * 64 * C), v);
      }
      if constexpr (EPI == kEpiDotAux) { red[r][0] = acc0; red[r][1] = acc1; }
      if constexpr (TS) { red[r][0] = acc0; red[r][1] = acc1; red[r][2] = acc2; red[r][3] = acc3; }
      if constexpr (EPI == kEpiResid) { red[r][0] = acc0; }
    }
  }
  if constexpr (EPI != kEpiNone) block_reduce_store_R<NV, R>(red, partials, r0, sched.nsb, bp.sb);
}

// ---------------------------------------------------------------------------
// Several right-hand sides on the matrix cores (FP16 storage).  A hop's SU(3)
// products for T right-hand sides at a site are one complex matrix product,
// U (3 x 3) times the 2T projected half-spinors (3 x 2T); in real form
// [[Re U, -Im U], [Im U, Re U]] times [Re h; Im h].  One 16 x 16 x 16 binary16
// matrix-core instruction takes two sites at once, block-diagonally: rows
// 8 s + 2 a + (re/im) of the output and columns 8 s + 2 b + (re/im) of K
// belong to site s of a wave's pair (colour 3 is padding), and its 16 columns
// are 8 right-hand sides times the two half-spinors (T = 12 or 16 takes two
// instructions per hop, sharing the link operand).  Lane l = 16 G + n feeds
// column n with K rows 4G .. 4G + 3 (site G / 2, colours 2 (G % 2) and
// 2 (G % 2) + 1) and receives the output rows of the same site and colours,
// so every lane projects, and later accumulates, only its own colour pair;
// the two half-spinors of a right-hand side sit in adjacent lanes and are
// exchanged after each product, so both lanes reconstruct the full
// four-spinor and each stores half of it.  Products are exact binary16
// products summed in FP32, as in the scalar FP16 path; the reconstruction
// is FP32.  Only the plain operator (no reduction epilogue) takes this form.
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// neighbour half index one hop along +mu (bwd false) or -mu (bwd true)
__device__ __forceinline__ int hop_neighbour_rt(const Geom& g, int h, const Coord& c, int mu, bool bwd) {
  if (mu == 0) {
    const int base = h - (c.x >> 1);
    const int xn = bwd ? ((c.x == 0) ? g.L[0] - 1 : c.x - 1) : ((c.x + 1 == g.L[0]) ? 0 : c.x + 1);
    return base + (xn >> 1);
  }
  const int cm = mu == 1 ? c.y : (mu == 2 ? c.z : c.t);
  const int st = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
  if (bwd) return (cm == 0) ? h + (g.L[mu] - 1) * st : h - st;
  return (cm + 1 == g.L[mu]) ? h - (g.L[mu] - 1) * st : h + st;
}


// binary16 value of a complex (re, im) pair scaled by a unit: 0 -> 1, 1 -> -1, 2 -> i, 3 -> -i
__device__ __forceinline__ h2v h_unit(h2v x, int code) {
  const h2v r = (code & 2) ? h2v{-x.y, x.x} : x;
  return (code == 1 || code == 3) ? -r : r;
}

template <typename S, int OP, int NC, int NE, bool EO>
__global__ __launch_bounds__(256) void k_dslash_mfma(Geom g, S* __restrict__ out, const S* __restrict__ in,
                                                     const S* __restrict__ U, double kappa,
                                                     const Scalars* __restrict__ scal, int ftz,
                                                     const S* __restrict__ cin, int tpar, int T, int mask) {
  static_assert(std::is_same<S, __half2>::value, "the matrix-core form is built for FP16 storage");
  constexpr bool DAG = (OP == kOpDdag || OP == kOpHdag);
  constexpr bool HOP_ONLY = (OP == kOpH || OP == kOpHdag);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n = lane & 15, G = lane >> 4;
  const int cg = G & 1;        // colour pair: (0, 1) or (2, padding)
  const int hh = n & 1;        // half-spinor of this lane's column
  const int r0 = blockIdx.y * T;
  const int nsite = EO ? g.Vh : 2 * g.Vh;
  const int pair = blockIdx.x * 4 + wid;
  const int my_site = 2 * pair + (G >> 1);              // the site of this lane's B / D rows
  const int a_site = 2 * pair + ((lane & 15) >> 3);     // the site of this lane's A rows
  const bool my_valid = my_site < nsite;
  // (par, h) of a site index; an index past the end maps to the parity's first site
  auto locate = [&](int sidx, int& par, int& h) {
    if (sidx >= nsite) sidx = sidx & 1;
    if (EO) {
      par = tpar;
      h = sidx;
    } else {
      par = sidx >= g.Vh;
      h = sidx - par * g.Vh;
    }
  };
  int mpar, mh, apar, ah;
  locate(my_site, mpar, mh);
  locate(a_site, apar, ah);
  const Coord mc = decode(g, mpar, mh), ac = decode(g, apar, ah);
  const size_t vs = EO ? (size_t)g.nb * 768 : spinor_elems(g);
  // A operand: row m = lane % 16 -> (site m / 8, colour row a, re/im ri); K group G -> (site G / 2, colours b0, b0 + 1)
  const int arow = lane & 15;
  const int a = (arow & 7) >> 1, ri = arow & 1, b0 = 2 * cg;
  const bool a_live = (arow >> 3) == (G >> 1) && a < 3;
  cx<float> acc[NC][4][2];  // [column group][spin][colour of the pair]
#pragma unroll
  for (int c = 0; c < NC; c++)
#pragma unroll
    for (int sp = 0; sp < 4; sp++)
#pragma unroll
      for (int k = 0; k < 2; k++) acc[c][sp][k] = cx<float>(0.f, 0.f);
  bool col_ok[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) col_ok[c] = (c * 8 + (n >> 1)) < T && my_valid;
  // skip right-hand sides whose solver stopped (uniform over a wave only per column, so no early exit)
#pragma unroll
  for (int c = 0; c < NC; c++)
    if (scal && col_ok[c] && !scal_live(scal[r0 + c * 8 + (n >> 1)], mask)) col_ok[c] = false;

#pragma unroll
  for (int hop = 0; hop < 8; hop++) {
    const int MU = hop >> 1;
    const bool BWD = hop & 1;
    const bool MINUS = BWD ? DAG : !DAG;
    // --- link of the A rows' site: U_mu(x) forward, U_mu(x - mu) backward (applied as U^dag)
    const int an = hop_neighbour_rt(g, ah, ac, MU, BWD);
    const int lp = BWD ? (apar ^ 1) : apar, lh = BWD ? an : ah;
    h2v u[9];
    {
      const S* lb = U + lk_block<NE>(g, MU, lp, lh);
      const int ll = lh & 63;
      if constexpr (NE == 6) {
        const typename Lay<S>::Gran q = *reinterpret_cast<const typename Lay<S>::Gran*>(lb + ll * 4);
#pragma unroll
        for (int k = 0; k < 4; k++) u[k] = h2_of(q.s[k]);
        const Pair<S> t = *reinterpret_cast<const Pair<S>*>(lb + 4 * 64 + ll * 2);
        u[4] = h2_of(t.s[0]);
        u[5] = h2_of(t.s[1]);
        h_third_row(u);
      } else {
        const typename Lay<S>::Gran q0 = *reinterpret_cast<const typename Lay<S>::Gran*>(lb + ll * 4);
        const typename Lay<S>::Gran q1 = *reinterpret_cast<const typename Lay<S>::Gran*>(lb + 64 * 4 + ll * 4);
#pragma unroll
        for (int k = 0; k < 4; k++) {
          u[k] = h2_of(q0.s[k]);
          u[4 + k] = h2_of(q1.s[k]);
        }
        u[8] = h2_of(lb[8 * 64 + ll]);
      }
    }
    // entries e_b = U[a][b] (forward) or conj(U[b][a]) (backward) for b = b0, b0 + 1
    h4v af = h4v{0, 0, 0, 0};
    if (a_live) {
#pragma unroll
      for (int j = 0; j < 2; j++) {
        const int b = b0 + j;
        h2v e = h2v{0, 0};
        if (b < 3) {
          const int idx = BWD ? 3 * b + a : 3 * a + b;
          h2v v = u[0];
#pragma unroll
          for (int k = 1; k < 9; k++) v = idx == k ? u[k] : v;
          e = BWD ? h2v{v.x, -v.y} : v;
        }
        // real form row ri: (Re e, -Im e) for ri = 0, (Im e, Re e) for ri = 1
        af[2 * j] = ri ? e.y : e.x;
        af[2 * j + 1] = ri ? e.x : -e.y;
      }
    }
    // --- B operand: this lane's half-spinor, colours of its pair, for each column group
    const int nn = hop_neighbour_rt(g, mh, mc, MU, BWD);
    const int npar = EO ? 0 : (mpar ^ 1);
    const S* sbase = in + sp_block(g, npar, nn) + (nn & 63) * 4;
    // spins and unit factor of this half (the projection of project_h)
    int sa, sb, code;
    if (MU == 0) { sa = hh; sb = 3 - hh; code = MINUS ? 2 : 3; }
    else if (MU == 1) { sa = hh; sb = 3 - hh; code = (MINUS != (hh == 1)) ? 0 : 1; }
    else if (MU == 2) { sa = hh; sb = 2 + hh; code = (MINUS != (hh == 1)) ? 2 : 3; }
    else { sa = sb = MINUS ? 2 + hh : hh; code = 0; }
    f4v d[NC];  // products: colours (a0, a1) of this lane's pair as (re, im, re, im)
#pragma unroll
    for (int c = 0; c < NC; c++) {
      h4v bf = h4v{0, 0, 0, 0};
      if (col_ok[c]) {
        const S* fb = sbase + (size_t)(c * 8 + (n >> 1)) * vs + (size_t)r0 * vs;
#pragma unroll
        for (int j = 0; j < 2; j++) {
          const int col = b0 + j;
          if (col < 3) {
            const int ka = 3 * sa + col, kb = 3 * sb + col;
            const h2v fa = h2_of(fb[(ka >> 2) * 256 + (ka & 3)]);
            const h2v fv = h2_of(fb[(kb >> 2) * 256 + (kb & 3)]);
            const h2v hv = fa + h_unit(fv, code);
            bf[2 * j] = hv.x;
            bf[2 * j + 1] = hv.y;
          }
        }
      }
      d[c] = __builtin_amdgcn_mfma_f32_16x16x16f16(af, bf, f4v{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    // --- exchange halves with the neighbouring lane and reconstruct (accumulate<MU, MINUS>)
#pragma unroll
    for (int c = 0; c < NC; c++) {
      f4v o;
#pragma unroll
      for (int q = 0; q < 4; q++) o[q] = __shfl_xor(d[c][q], 1, 64);
      const f4v u1 = hh ? o : d[c], u2 = hh ? d[c] : o;  // half 1 and half 2, colours (a0, a1) as (re, im, re, im)
#pragma unroll
      for (int k = 0; k < 2; k++) {
        const float x1 = u1[2 * k], y1 = u1[2 * k + 1], x2 = u2[2 * k], y2 = u2[2 * k + 1];
        auto add = [&](int sp, float xr, float xi) {
          acc[c][sp][k].re += xr;
          acc[c][sp][k].im += xi;
        };
        if (MU == 3) {
          if (MINUS) { add(2, x1, y1); add(3, x2, y2); }
          else { add(0, x1, y1); add(1, x2, y2); }
        } else {
          add(0, x1, y1);
          add(1, x2, y2);
          if (MU == 0) {
            if (MINUS) { add(2, y2, -x2); add(3, y1, -x1); }   // -i u2, -i u1
            else { add(2, -y2, x2); add(3, -y1, x1); }         //  i u2,  i u1
          } else if (MU == 1) {
            if (MINUS) { add(2, -x2, -y2); add(3, x1, y1); }
            else { add(2, x2, y2); add(3, -x1, -y1); }
          } else {
            if (MINUS) { add(2, y1, -x1); add(3, -y2, x2); }   // -i u1,  i u2
            else { add(2, -y1, x1); add(3, y2, -x2); }         //  i u1, -i u2
          }
        }
      }
    }
  }
  // --- output: this lane's colours, spins (0, 1) for half 0 and (2, 3) for half 1
  const float k = (float)kappa;
#pragma unroll
  for (int c = 0; c < NC; c++) {
    if (!col_ok[c]) continue;
    const size_t fo = (size_t)(r0 + c * 8 + (n >> 1)) * vs + sp_block(g, EO ? 0 : mpar, mh) + (mh & 63) * 4;
    const S* cb = (EO ? cin : in) + fo;
    S* ob = out + fo;
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int sp = 2 * hh + q;
#pragma unroll
      for (int j = 0; j < 2; j++) {
        const int col = b0 + j;
        if (col >= 3) continue;
        const int kk = 3 * sp + col;
        const int off = (kk >> 2) * 256 + (kk & 3);
        // acc holds spins by index; select this lane's spin without indexing registers at run time
        const float xr = hh ? acc[c][2 + q][j].re : acc[c][q][j].re;
        const float xi = hh ? acc[c][2 + q][j].im : acc[c][q][j].im;
        cx<float> o(xr, xi);
        if constexpr (!HOP_ONLY) {
          const cx<float> ctr = Traits<S>::load(cb + off);
          o = cx<float>(ctr.re - k * xr, ctr.im - k * xi);
        }
        ob[off] = Traits<S>::pack(o, ftz);
      }
    }
  }
}

// One translation unit per storage precision (QCD_DSLASH_PREC = 0, 1, 2, 3 for
// FP64, FP32, FP16, BF16) keeps the kernel instantiations of a build parallel; the
// FP16 unit also holds the precision-independent helpers and the dispatcher.
#ifndef QCD_DSLASH_PREC
#define QCD_DSLASH_PREC 2
#endif

template <typename S, int DEPTH, int OCC, int T, int NE>
static void launch_dslash_v(const Geom& g, const DslashSched& sc, int op, int epi, void* out, const void* in,
                            const void* U, double kappa, const void* aux, double* partials, const Scalars* scal,
                            int ftz, const void* cin, int eo_par, hipStream_t st, int mask) {
  dim3 grid(sc.nsb * sc.ntiles), block(256);
  S* o = (S*)out;
  const S* i = (const S*)in;
  const S* u = (const S*)U;
  const S* x = (const S*)aux;
  const S* ci = (const S*)cin;
  if (eo_par >= 0) {  // one parity: D form (centre from cin) or H, the epilogues the solvers use
#define QCD_LAUNCH_EO(OPV, EPIV)                                                                                     \
  do {                                                                                                               \
    if (T == 1 && sc.ntiles == 1)                                                                                    \
      hipLaunchKernelGGL((k_dslash<S, OPV, EPIV, DEPTH, OCC, T, NE, true, T == 1>), grid, block, 0, st, g, sc, o, i, \
                         u, kappa, x, partials, scal, ftz, ci, eo_par, mask);                                        \
    else                                                                                                             \
      hipLaunchKernelGGL((k_dslash<S, OPV, EPIV, DEPTH, OCC, T, NE, true, false>), grid, block, 0, st, g, sc, o, i,  \
                         u, kappa, x, partials, scal, ftz, ci, eo_par, mask);                                        \
  } while (0)
    if (op == kOpH) QCD_LAUNCH_EO(kOpH, kEpiNone);
    else if (epi == kEpiNone) QCD_LAUNCH_EO(kOpD, kEpiNone);
    else if (epi == kEpiDotAux) QCD_LAUNCH_EO(kOpD, kEpiDotAux);
    else if (epi == kEpiTS) QCD_LAUNCH_EO(kOpD, kEpiTS);
    else if (epi == kEpiTSAux) {  // the network-preconditioned Schur operator: FP16 only
      if constexpr (std::is_same<S, __half2>::value) QCD_LAUNCH_EO(kOpD, kEpiTSAux);
    } else if (epi == kEpiRecon) {
      if constexpr (std::is_same<S, double2>::value && T == 1) QCD_LAUNCH_EO(kOpD, kEpiRecon);
    } else QCD_LAUNCH_EO(kOpD, kEpiResid);
#undef QCD_LAUNCH_EO
    return;
  }
#define QCD_LAUNCH(OPV, EPIV)                                                                                          \
  hipLaunchKernelGGL((k_dslash<S, OPV, EPIV, DEPTH, OCC, T, NE, false, false>), grid, block, 0, st, g, sc, o, i, u, kappa, \
                     x, partials, scal, ftz, nullptr, 0, mask)
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
  } else if (epi == kEpiTSAux) {
    QCD_LAUNCH(kOpD, kEpiTSAux);
  } else {
    QCD_LAUNCH(kOpD, kEpiResid);
  }
#undef QCD_LAUNCH
}

template <typename S, int NE, int DEPTH>
static void launch_dslash_lds_eo(const Geom& g, const DslashSched& sc, int op, int epi, void* out, const void* in,
                                 const void* U, double kappa, const void* aux, double* partials, const Scalars* scal,
                                 int ftz, const void* cin, int eo_par, hipStream_t st, int mask) {
  const dim3 grid(sc.nsb * sc.ntiles), block(256);
#define QCD_LDS_EO(OPV, EPIV)                                                                                    \
  hipLaunchKernelGGL((k_dslash_lds_eo<S, OPV, EPIV, DEPTH, NE>), grid, block, 0, st, g, sc, (S*)out, (const S*)in, \
                     (const S*)U, kappa, (const S*)aux, partials, scal, ftz, (const S*)cin, eo_par, mask)
  if (op == kOpH) QCD_LDS_EO(kOpH, kEpiNone);
  else if (epi == kEpiNone) QCD_LDS_EO(kOpD, kEpiNone);
  else if (epi == kEpiDotAux) QCD_LDS_EO(kOpD, kEpiDotAux);
  else if (epi == kEpiTS) QCD_LDS_EO(kOpD, kEpiTS);
  else if (epi == kEpiTSAux) {
    if constexpr (std::is_same<S, __half2>::value) QCD_LDS_EO(kOpD, kEpiTSAux);
  } else QCD_LDS_EO(kOpD, kEpiResid);
#undef QCD_LDS_EO
}

template <typename S, int NE, int DEPTH>
static void launch_dslash_lds(const Geom& g, const DslashSched& sc, int op, void* out, const void* in, const void* U,
                              double kappa, int ftz, hipStream_t st) {
  const dim3 grid(sc.nsb), block(256);
#define QCD_LDS(OPV)                                                                                           \
  hipLaunchKernelGGL((k_dslash_lds<S, OPV, DEPTH, NE>), grid, block, 0, st, g, sc, (S*)out, (const S*)in, (const S*)U, \
                     kappa, ftz)
  switch (op) {
    case kOpD: QCD_LDS(kOpD); break;
    case kOpH: QCD_LDS(kOpH); break;
    case kOpDdag: QCD_LDS(kOpDdag); break;
    default: QCD_LDS(kOpHdag); break;
  }
#undef QCD_LDS
}

template <typename S, int T, int NE>
static void launch_dslash_tile(const Geom& g, const DslashTune& tune, int op, int epi, int n, void* out,
                               const void* in, const void* U, double kappa, const void* aux, double* partials,
                               const Scalars* scal, int ftz, const void* cin, int eo_par, hipStream_t st, int mask) {
  const DslashSched sc = make_sched(g, tune.sched, T, n, eo_par >= 0);
  if constexpr (T == 1) {
    const bool lds = tune.variant == 6 || tune.variant == 7;
    // variants 6 and 7: x and y neighbours staged in LDS; the full-lattice form
    // (16-bit storage: 24 KB per block; plain operator, one right-hand side) ...
    if constexpr (sizeof(S) == 4) {
      if (lds && n == 1 && eo_par < 0 && epi == kEpiNone && !scal && lds_form_applies(g)) {
        if (tune.variant == 7)
          launch_dslash_lds<S, NE, 2>(g, sc, op, out, in, U, kappa, ftz, st);
        else
          launch_dslash_lds<S, NE, 1>(g, sc, op, out, in, U, kappa, ftz, st);
        return;
      }
    }
    // ... and the one-parity form for the even-odd solvers (the epilogues they use)
    if (lds && eo_par >= 0 && epi != kEpiRecon && (op == kOpH || op == kOpD) && n == 1 &&
        lds_eo_form_applies<S>(g) && sc.H == 256) {
      if (sizeof(S) == 4 && tune.variant == 7)
        launch_dslash_lds_eo<S, NE, 2>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st,
                                       mask);
      else
        launch_dslash_lds_eo<S, NE, 1>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st,
                                       mask);
      return;
    }
  }
  if constexpr (T > 1) {  // multi-RHS tiles are built in the default variant only
    launch_dslash_v<S, 1, 2, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
    return;
  }
  switch (tune.variant) {
    case 1:
    case 6: launch_dslash_v<S, 2, 2, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask); break;
    case 2: launch_dslash_v<S, 0, 3, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask); break;
    case 3: launch_dslash_v<S, 1, 3, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask); break;
    case 4: launch_dslash_v<S, 0, 4, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask); break;
    case 5: launch_dslash_v<S, 1, 4, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask); break;
    default: launch_dslash_v<S, 1, 2, T, NE>(g, sc, op, epi, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask); break;
  }
}

template <typename S, int R, int NE>
static void launch_dslash_mr(const Geom& g, const DslashTune& tune, int op, int epi, int n, void* out, const void* in,
                             const void* U, double kappa, const void* aux, double* partials, const Scalars* scal,
                             int ftz, const void* cin, int eo_par, hipStream_t st, int mask) {
  const DslashSched sc = make_sched(g, tune.sched, 1, n / R, eo_par >= 0);
  dim3 grid(sc.nsb * sc.ntiles), block(256);
  S* o = (S*)out;
  const S* i = (const S*)in;
  const S* u = (const S*)U;
  const S* x = (const S*)aux;
  const S* ci = (const S*)cin;
  if (eo_par >= 0) {
#define QCD_LAUNCH_EO(OPV, EPIV)                                                                                 \
  hipLaunchKernelGGL((k_dslash_mr<S, OPV, EPIV, R, NE, true>), grid, block, 0, st, g, sc, o, i, u, kappa, x, partials, \
                     scal, ftz, ci, eo_par, mask)
    if (op == kOpH) QCD_LAUNCH_EO(kOpH, kEpiNone);
    else if (epi == kEpiNone) QCD_LAUNCH_EO(kOpD, kEpiNone);
    else if (epi == kEpiDotAux) QCD_LAUNCH_EO(kOpD, kEpiDotAux);
    else if (epi == kEpiTS) QCD_LAUNCH_EO(kOpD, kEpiTS);
    else if (epi == kEpiTSAux) {
      if constexpr (std::is_same<S, __half2>::value) QCD_LAUNCH_EO(kOpD, kEpiTSAux);
    } else QCD_LAUNCH_EO(kOpD, kEpiResid);
#undef QCD_LAUNCH_EO
    return;
  }
#define QCD_LAUNCH(OPV, EPIV)                                                                                     \
  hipLaunchKernelGGL((k_dslash_mr<S, OPV, EPIV, R, NE, false>), grid, block, 0, st, g, sc, o, i, u, kappa, x, partials, \
                     scal, ftz, nullptr, 0, mask)
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
  } else if (epi == kEpiTSAux) {
    QCD_LAUNCH(kOpD, kEpiTSAux);
  } else {
    QCD_LAUNCH(kOpD, kEpiResid);
  }
#undef QCD_LAUNCH
}

// The matrix-core form: grid.x covers the site pairs (four per block), grid.y the tiles of T right-hand sides.
template <int NE>
static void launch_dslash_mfma(const Geom& g, int op, int n, void* out, const void* in, const void* U,
                               double kappa, const Scalars* scal, int ftz, const void* cin, int eo_par,
                               hipStream_t st, int mask) {
  const int T = mfma_rhs_tile(n);
  const bool eo = eo_par >= 0;
  const int nsite = eo ? g.Vh : 2 * g.Vh;
  const int npair = (nsite + 1) / 2;
  const dim3 grid((npair + 3) / 4, n / T), block(256);
  __half2* o = (__half2*)out;
  const __half2* i = (const __half2*)in;
  const __half2* u = (const __half2*)U;
  const __half2* ci = (const __half2*)cin;
  const int tp = eo ? eo_par : 0;
#define QCD_MFMA(OPV, EOV)                                                                                        \
  do {                                                                                                            \
    if (T > 8)                                                                                                    \
      hipLaunchKernelGGL((k_dslash_mfma<__half2, OPV, 2, NE, EOV>), grid, block, 0, st, g, o, i, u, kappa, scal, ftz, \
                         ci, tp, T, mask);                                                                        \
    else                                                                                                          \
      hipLaunchKernelGGL((k_dslash_mfma<__half2, OPV, 1, NE, EOV>), grid, block, 0, st, g, o, i, u, kappa, scal, ftz, \
                         ci, tp, T, mask);                                                                        \
  } while (0)
  if (eo) {
    if (op == kOpH) QCD_MFMA(kOpH, true);
    else QCD_MFMA(kOpD, true);
  } else {
    switch (op) {
      case kOpD: QCD_MFMA(kOpD, false); break;
      case kOpH: QCD_MFMA(kOpH, false); break;
      case kOpDdag: QCD_MFMA(kOpDdag, false); break;
      default: QCD_MFMA(kOpHdag, false); break;
    }
  }
#undef QCD_MFMA
}

template <typename S, int NE>
static void launch_dslash_r(const Geom& g, const DslashTune& tune, int op, int epi, int n, void* out, const void* in,
                            const void* U, double kappa, const void* aux, double* partials, const Scalars* scal,
                            int ftz, const void* cin, int eo_par, hipStream_t st, int mask) {
  if constexpr (std::is_same<S, __half2>::value) {
    // the matrix-core form, when chosen, for the plain operator of a tileable number of right-hand sides
    if (tune.rhs_tile == kRhsTileMfma && epi == kEpiNone && mfma_rhs_tile(n) > 0) {
      launch_dslash_mfma<NE>(g, op, n, out, in, U, kappa, scal, ftz, cin, eo_par, st, mask);
      return;
    }
  }
  const int R = reg_tile_for(tune, n);
  if (R == 4) return launch_dslash_mr<S, 4, NE>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  if (R == 3) return launch_dslash_mr<S, 3, NE>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  if (R == 2) return launch_dslash_mr<S, 2, NE>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  const int T = rhs_tile_for(tune, n);
  if (T == 4)
    launch_dslash_tile<S, 4, NE>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  else if (T == 2)
    launch_dslash_tile<S, 2, NE>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  else
    launch_dslash_tile<S, 1, NE>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}

template <typename S>
static void launch_dslash_t(const Geom& g, const DslashTune& tune, int op, int epi, int n, void* out, const void* in,
                            const void* U, double kappa, const void* aux, double* partials, const Scalars* scal,
                            int ftz, const void* cin, int eo_par, hipStream_t st, int mask) {
  if (tune.recon)
    launch_dslash_r<S, 6>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  else
    launch_dslash_r<S, 9>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}

#define QCD_DSLASH_ARGS                                                                                          \
  const Geom &g, const DslashTune &tune, int op, int epi, int n, void *out, const void *in, const void *U, \
      double kappa, const void *aux, double *partials, const Scalars *scal, int ftz, const void *cin, int eo_par, \
      hipStream_t st, int mask
void launch_dslash_f64(QCD_DSLASH_ARGS);
void launch_dslash_f32(QCD_DSLASH_ARGS);
void launch_dslash_f16(QCD_DSLASH_ARGS);
void launch_dslash_bf16(QCD_DSLASH_ARGS);

#if QCD_DSLASH_PREC == 0
void launch_dslash_f64(QCD_DSLASH_ARGS) {
  launch_dslash_t<double2>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}
#elif QCD_DSLASH_PREC == 1
void launch_dslash_f32(QCD_DSLASH_ARGS) {
  launch_dslash_t<float2>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}
#elif QCD_DSLASH_PREC == 3
void launch_dslash_bf16(QCD_DSLASH_ARGS) {
  launch_dslash_t<bf2>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}
#else
void launch_dslash_f16(QCD_DSLASH_ARGS) {
  launch_dslash_t<__half2>(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}

int rhs_tile_for(const DslashTune& tune, int n) {
  int T = tune.rhs_tile;
  if (T <= 0) T = 1;  // measured fastest at 32^3 x 64 with 12 right-hand sides (T = 2 ties, T = 4 is slower)
  if (T != 1 && T != 2 && T != 4) T = 1;
  if (n % T) T = 1;
  return T;
}

int reg_tile_for(const DslashTune& tune, int n) {
  const int R = -tune.rhs_tile;
  return (R >= 2 && R <= 4 && n % R == 0) ? R : 1;
}

// The automatic choice (rhs_tile = 0) for n right-hand sides in precision
// prec: FP16 is bound by instruction issue per site-RHS, so several
// right-hand sides per thread pay (3 measured best at 32^3 x 64, then 2); FP32
// and FP64 are bound by bandwidth and keep one per thread.
DslashTune resolve_rhs_tile(const DslashTune& tune, int prec, int n) {
  DslashTune t = tune;
  if (t.rhs_tile == 0 && prec == kFP16 && n > 1) t.rhs_tile = (n % 3 == 0) ? -3 : ((n % 2 == 0) ? -2 : 1);
  return t;
}

DslashSched make_sched(const Geom& g, int mode, int T, int n, bool eo) {
  DslashSched s;
  s.H = (eo ? 256 : 128) / T;  // half sites of one parity (eo) or of each parity per block
  s.nsb = (g.Vh + s.H - 1) / s.H;
  s.ntiles = n / T;
  s.mode = 0;
  s.Lz = g.L[2];
  s.Lt = g.L[3];
  s.bp = 1;
  s.zc = 1;
  s.sub = 1;
  const int plane = g.Lxh * g.L[1];
  if (mode == 4) {
    // XCD slabs of Lt/8 time slices, each swept in z order
    if (plane % s.H == 0 && g.L[3] % 8 == 0) {
      s.mode = 4;
      s.bp = plane / s.H;
      s.zc = g.L[3] / 8;
    }
    return s;
  }
  // mode m = 1..3: XCD slabs of Lz/8 planes, each swept as 2^(m-1) sub-slabs in t order
  const int sub = mode >= 1 ? 1 << (mode - 1) : 1;
  if (mode >= 1 && plane % s.H == 0 && g.L[2] % (8 * sub) == 0) {
    s.mode = mode;
    s.bp = plane / s.H;
    s.zc = g.L[2] / 8;
    s.sub = sub;
  }
  return s;
}

int dslash_partial_rows(const Geom& g, const DslashTune& tune, int n, bool eo) {
  const int T = rhs_tile_for(tune, n);
  const int H = (eo ? 256 : 128) / T;
  return (g.Vh + H - 1) / H;
}

void launch_dslash(int prec, const Geom& g, const DslashTune& tune_in, int op, int epi, int n, void* out,
                   const void* in, const void* U, double kappa, const void* aux, double* partials, const Scalars* scal,
                   int ftz, hipStream_t st, const void* cin, int eo_par, int mask) {
  DslashTune tune = resolve_rhs_tile(tune_in, prec, n);
  if (epi == kEpiRecon) tune.rhs_tile = 1;  // built for one right-hand side per thread only
  if (prec == kFP64)
    launch_dslash_f64(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  else if (prec == kFP32)
    launch_dslash_f32(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  else if (prec == kBF16)
    launch_dslash_bf16(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
  else
    launch_dslash_f16(g, tune, op, epi, n, out, in, U, kappa, aux, partials, scal, ftz, cin, eo_par, st, mask);
}
#endif
#undef QCD_DSLASH_ARGS

}  // namespace qcd
