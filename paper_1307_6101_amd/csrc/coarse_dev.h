// Device building blocks of the coarse block stencil and workgroup
// reductions (shared by the coarse apply, SAP, transfer and Galerkin kernels).
#pragma once

#include "coarse.h"

namespace ddamg {

// ---------------------------------------------------------------------------
// workgroup reductions
// ---------------------------------------------------------------------------
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

// ---------------------------------------------------------------------------
// stencil rows
// ---------------------------------------------------------------------------
// row i of B_k(x) v(y), summed over j: forward-stored block M (row-major d x d)
template <typename T>
__device__ inline C<T> row_fwd(const C<T>* __restrict__ M, const C<T>* __restrict__ v, int i, int d) {
  C<T> acc = czero<T>();
  const C<T>* m = M + (size_t)i * d;
  for (int j = 0; j < d; ++j) cfma(acc, m[j], v[j]);
  return acc;
}
// row i of G5 F^H G5 v: g_i sum_j g_j conj(F[j][i]) v_j
template <typename T>
__device__ inline C<T> row_bwd(const C<T>* __restrict__ F, const C<T>* __restrict__ v, int i, int d) {
  const int h = d >> 1;
  C<T> a = czero<T>(), b = czero<T>();
  for (int j = 0; j < h; ++j) cjfma(a, F[(size_t)j * d + i], v[j]);
  for (int j = h; j < d; ++j) cjfma(b, F[(size_t)j * d + i], v[j]);
  C<T> r = csub(a, b);
  return i < h ? r : mk<T>(-r.x, -r.y);
}

// full stencil row: (D v)(site)[i]
template <typename T>
__device__ inline C<T> stencil_row(const CoarseOpView<T>& op, const C<T>* __restrict__ v, int site, int i) {
  const int d = op.d;
  const size_t bsz = (size_t)d * d;
  const C<T>* Ds = op.D + (size_t)site * 5 * bsz;
  C<T> acc = row_fwd<T>(Ds, v + (size_t)site * d, i, d);
  for (int mu = 0; mu < 4; ++mu) {
    const int nf = op.nbr[site * 8 + 2 * mu];
    acc = cadd(acc, row_fwd<T>(Ds + (1 + mu) * bsz, v + (size_t)nf * d, i, d));
    const int nb = op.nbr[site * 8 + 2 * mu + 1];
    acc = cadd(acc, row_bwd<T>(op.D + ((size_t)nb * 5 + 1 + mu) * bsz, v + (size_t)nb * d, i, d));
  }
  return acc;
}

}  // namespace ddamg
