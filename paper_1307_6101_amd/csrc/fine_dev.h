// Device building blocks of the fine-lattice stencil (shared by the
// Wilson-clover, SAP and Galerkin kernels).  See fine.hip for the spin
// projection scheme.
#pragma once

#include "fine.h"

namespace ddamg {

// ---------------------------------------------------------------------------
// stencil building blocks
// ---------------------------------------------------------------------------
// multiply by k-th power of i: 0: 1, 1: i, 2: -1, 3: -i
template <int K, typename V> __device__ inline V mul_ik(V a) {
  if constexpr (K == 0) return a;
  else if constexpr (K == 1) return cmuli(a);
  else if constexpr (K == 2) { a.x = -a.x; a.y = -a.y; return a; }
  else return cmulmi(a);
}

template <int MU> struct Proj;
template <> struct Proj<0> { static constexpr int J0 = 3, K0 = 1, J1 = 2, K1 = 1; };
template <> struct Proj<1> { static constexpr int J0 = 3, K0 = 0, J1 = 2, K1 = 2; };
template <> struct Proj<2> { static constexpr int J0 = 2, K0 = 1, J1 = 3, K1 = 3; };
template <> struct Proj<3> { static constexpr int J0 = 2, K0 = 2, J1 = 3, K1 = 2; };

// project the spinor psi (12 components) for the hop in direction MU
// (FWD: (1-g_mu), else (1+g_mu)), multiply by the link (U or U^H), and add
// the rebuilt spinor to acc.
template <typename T, int MU, bool FWD>
__device__ inline void hop_apply(const C<T> psi[12], const C<T> u[9], C<T> acc[12]) {
  using P = Proj<MU>;
  constexpr int k0 = FWD ? P::K0 : (P::K0 + 2) & 3;
  constexpr int k1 = FWD ? P::K1 : (P::K1 + 2) & 3;
  C<T> h[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h[a] = cadd(psi[a], mul_ik<k0>(psi[P::J0 * 3 + a]));
    h[3 + a] = cadd(psi[3 + a], mul_ik<k1>(psi[P::J1 * 3 + a]));
  }
  C<T> chi[6];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C<T> v = czero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (FWD) cfma(v, u[a * 3 + b], h[s * 3 + b]);
        else cjfma(v, u[b * 3 + a], h[s * 3 + b]);
      }
      chi[s * 3 + a] = v;
    }
  constexpr int c0 = (4 - k0) & 3, c1 = (4 - k1) & 3;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] = cadd(acc[a], chi[a]);
    acc[3 + a] = cadd(acc[3 + a], chi[3 + a]);
    acc[P::J0 * 3 + a] = cadd(acc[P::J0 * 3 + a], mul_ik<c0>(chi[a]));
    acc[P::J1 * 3 + a] = cadd(acc[P::J1 * 3 + a], mul_ik<c1>(chi[3 + a]));
  }
}

// Workgroups are dealt to the eight XCDs round-robin (workgroup i runs on XCD
// i mod 8), each with its own L2.  Map workgroup i to a logical index so that
// every XCD processes one contiguous slab of blocks: lattice neighbours then
// share an L2 instead of being fetched again by another XCD.
__device__ inline int xcd_slab_index(int bid, int nwg) {
  if (nwg % 8 != 0) return bid;
  return (bid & 7) * (nwg >> 3) + (bid >> 3);
}
// The same for a batch of nb fields over a one-dimensional grid of gx * nb
// workgroups: each XCD takes one slab of blocks and runs the nb fields of a
// block chunk back to back, so the operator data of the chunk is fetched
// into that XCD's L2 once for all of them.  Sets the workgroup's block-chunk
// index x and field r.
__device__ inline void xcd_slab_rhs(int bid, int gx, int nb, int& x, int& r) {
  if (gx % 8 != 0) {
    x = bid % gx;
    r = bid / gx;
    return;
  }
  const int k = bid >> 3;
  x = (bid & 7) * (gx >> 3) + k / nb;
  r = k % nb;
}

template <typename T, typename S = C<T>>
__device__ inline void load_spinor(const S* __restrict__ f, int blk, int loc, C<T> v[12]) {
  const S* p = f + (long long)blk * 192 + loc;
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = ldc<T, S>(p[c * 16]);
}
// A fine spinor field of storage V: complex numbers of the arithmetic
// precision (V = C<T>), or FP16 (V = __half2), each site's 12 components
// divided by their largest |re|, |im|, which is kept in FP32 per site
// ([field][nblk * 16], native site order) next to them.  load_site /
// store_site read and write one site in either form; the scale pointer is
// not used for V = C<T>.
template <typename T, typename V>
__device__ inline void load_site(const V* __restrict__ f, const float* __restrict__ sc, int blk, int loc,
                                 C<T> v[12]) {
  load_spinor<T, V>(f, blk, loc, v);
  if constexpr (std::is_same<V, __half2>::value) {
    const T m = sc[(long long)blk * 16 + loc];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      v[c].x *= m;
      v[c].y *= m;
    }
  }
}
template <typename T, typename V>
__device__ inline void store_site(V* __restrict__ f, float* __restrict__ sc, int blk, int loc, const C<T> v[12]) {
  V* p = f + (long long)blk * 192 + loc;
  if constexpr (std::is_same<V, __half2>::value) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf((float)v[c].x), fabsf((float)v[c].y)));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    sc[(long long)blk * 16 + loc] = m;
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c * 16] = __floats2half2_rn((float)v[c].x * inv, (float)v[c].y * inv);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c * 16] = v[c];
  }
}

template <typename T, typename S = C<T>>
__device__ inline void load_link(const S* __restrict__ U, int blk, int loc, int mu, C<T> u[9]) {
  const S* p = U + (long long)blk * 576 + mu * 144 + loc;
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = ldc<T, S>(p[k * 16]);
}

// out = A(x) v for the packed clover of one site (both chiralities); get(e)
// returns entry e = 0..35 as C<T>: per chirality 3 packed real diagonal
// pairs, then the 15 upper off-diagonal entries row by row
// one chirality block h of the clover: o = A_h w (6 components each)
template <typename T, typename G>
__device__ inline void clover_block(int h, G&& get, const C<T>* w, C<T>* o) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const C<T> d = get(h * 18 + k);
    o[2 * k] = cscale(w[2 * k], d.x);
    o[2 * k + 1] = cscale(w[2 * k + 1], d.y);
  }
  int e = 3;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a + 1; b < 6; ++b) {
      const C<T> m = get(h * 18 + e);
      ++e;
      cfma(o[a], m, w[b]);
      cjfma(o[b], m, w[a]);
    }
}

template <typename T, typename G>
__device__ inline void clover_mul(G&& get, const C<T> v[12], C<T> out[12]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) clover_block<T>(h, get, v + 6 * h, out + 6 * h);
}

template <typename T, typename S = C<T>>
__device__ inline void clover_apply(const S* __restrict__ A, int blk, int loc, const C<T> v[12],
                                    C<T> out[12]) {
  const S* p = A + (long long)blk * 576 + loc;
  clover_mul<T>([&](int e) { return ldc<T, S>(p[e * 16]); }, v, out);
}

}  // namespace ddamg
