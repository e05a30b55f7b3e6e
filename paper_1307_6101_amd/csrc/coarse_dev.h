// Device building blocks of the coarse block stencil and workgroup
// reductions (shared by the coarse apply, SAP, transfer and Galerkin kernels).
#pragma once

#include <type_traits>

#include "coarse.h"

namespace ddamg {

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum of NV values over the whole workgroup; every thread gets the result.
// scratch: >= 16 * NV elements of LDS.
template <typename T, int NV>
__device__ inline void wg_sum(T (&v)[NV], T* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) scratch[wave * NV + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T s = 0;
    for (int w = 0; w < nw; ++w) s += scratch[w * NV + k];
    v[k] = s;
  }
  __syncthreads();
}

// Row i of a column-major d x d block times a vector held in LDS (every lane
// reads the same v[j], a broadcast): acc += sum_j M[j*d + i] v[j].
// NCH = ceil(d / 8) is a compile-time bound, so all d loads of the row are
// issued before the first multiply: one memory round trip per block.
// GMAX caps the chunks loaded at once (FP64 rows at most three chunks).
template <typename T, int NCH, int GMAX = 8>
__device__ inline void colmajor_row(const C<T>* __restrict__ M, const C<T>* v, int i, int d, C<T>& acc) {
  constexpr int G0 = sizeof(T) == 4 ? NCH : (NCH < 3 ? NCH : 3);
  constexpr int G = G0 < GMAX ? G0 : GMAX;
  C<T> a[4] = {czero<T>(), czero<T>(), czero<T>(), czero<T>()};
#pragma unroll 1
  for (int c0 = 0; c0 < NCH; c0 += G) {
    C<T> m[8 * G];
#pragma unroll
    for (int u = 0; u < 8 * G; ++u) {
      const int j = 8 * c0 + u;
      m[u] = j < d ? M[(size_t)j * d + i] : czero<T>();
    }
#pragma unroll
    for (int u = 0; u < 8 * G; ++u)
      if (8 * c0 + u < d) cfma(a[u & 3], m[u], v[8 * c0 + u]);
  }
  acc = cadd(acc, cadd(cadd(a[0], a[1]), cadd(a[2], a[3])));
}

// run f(std::integral_constant<int, NCH>) for NCH = ceil(d / 8), d <= 64
template <typename F>
inline void with_nch(int d, F&& f) {
  switch ((d + 7) / 8) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: throw Error(-1, "coarse levels support at most 64 components per site");
  }
}

}  // namespace ddamg
