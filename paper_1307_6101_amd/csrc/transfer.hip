// Interpolation kernels: restriction P^H, prolongation P, block
// orthonormalisation of the test vectors and the FP64 Galerkin products.
#include "coarse_dev.h"
#include "fine_dev.h"
#include "transfer.h"

namespace ddamg {

AggTables make_fine_agg(const FineGeom& g, const int agg[4]) {
  AggTables a;
  a.nagg = 1;
  a.asz = 1;
  int bpa[4], na[4];
  for (int mu = 0; mu < 4; ++mu) {
    a.agg[mu] = agg[mu];
    DD_REQUIRE(agg[mu] % 2 == 0 && g.dims[mu] % agg[mu] == 0,
               "fine aggregates must be even and tile the lattice");
    na[mu] = g.dims[mu] / agg[mu];
    bpa[mu] = agg[mu] / 2;
    a.cdims[mu] = na[mu];
    a.nagg *= na[mu];
    a.asz *= agg[mu];
  }
  const int nbpa = a.asz / 16;
  a.members.resize((size_t)a.nagg * nbpa);
  a.member_agg.resize(g.nblk);
  for (int A = 0; A < a.nagg; ++A) {
    int c[4], r = A;
    for (int mu = 0; mu < 4; ++mu) { c[mu] = r % na[mu]; r /= na[mu]; }
    for (int j = 0; j < nbpa; ++j) {
      int l[4], rr = j;
      for (int mu = 0; mu < 4; ++mu) { l[mu] = rr % bpa[mu]; rr /= bpa[mu]; }
      int b[4];
      for (int mu = 0; mu < 4; ++mu) b[mu] = c[mu] * bpa[mu] + l[mu];
      int blk = block_encode(g.nb, b);
      a.members[(size_t)A * nbpa + j] = blk;
      a.member_agg[blk] = A;
    }
  }
  return a;
}

AggTables make_coarse_agg(const CoarseGeom& g, const int agg[4]) {
  AggTables a;
  a.nagg = 1;
  a.asz = 1;
  int na[4];
  for (int mu = 0; mu < 4; ++mu) {
    a.agg[mu] = agg[mu];
    DD_REQUIRE(agg[mu] >= 1 && g.dims[mu] % agg[mu] == 0, "aggregates must tile the lattice");
    na[mu] = g.dims[mu] / agg[mu];
    a.cdims[mu] = na[mu];
    a.nagg *= na[mu];
    a.asz *= agg[mu];
  }
  a.members.resize((size_t)a.nagg * a.asz);
  a.member_agg.resize(g.V);
  for (int A = 0; A < a.nagg; ++A) {
    int c[4], r = A;
    for (int mu = 0; mu < 4; ++mu) { c[mu] = r % na[mu]; r /= na[mu]; }
    for (int j = 0; j < a.asz; ++j) {
      int l[4], rr = j;
      for (int mu = 0; mu < 4; ++mu) { l[mu] = rr % agg[mu]; rr /= agg[mu]; }
      int x[4];
      for (int mu = 0; mu < 4; ++mu) x[mu] = c[mu] * agg[mu] + l[mu];
      int s = x[0] + g.dims[0] * (x[1] + g.dims[1] * (x[2] + g.dims[2] * x[3]));
      a.members[(size_t)A * a.asz + j] = s;
      a.member_agg[s] = A;
    }
  }
  return a;
}

// ---------------------------------------------------------------------------
// per-(aggregate, chirality) reduction of 2N partial sums: each thread holds
// for coarse row k the pair (sigma=0, sigma=1) of complex partials, which are
// wave-reduced and collected in LDS as red[wave][k][4].
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void stash4(T* red, int N, int k, T a, T b, T c, T d) {
  a = wave_sum(a); b = wave_sum(b); c = wave_sum(c); d = wave_sum(d);
  if ((threadIdx.x & 63) == 0) {
    T* r = red + ((threadIdx.x >> 6) * N + k) * 4;
    r[0] = a; r[1] = b; r[2] = c; r[3] = d;
  }
}
// after a barrier: sum over waves of entry (sigma, k)
template <typename T>
__device__ inline C<T> collect(const T* red, int N, int sigma, int k) {
  const int nw = (blockDim.x + 63) >> 6;
  T re = 0, im = 0;
  for (int w = 0; w < nw; ++w) {
    re += red[(w * N + k) * 4 + 2 * sigma];
    im += red[(w * N + k) * 4 + 2 * sigma + 1];
  }
  return mk<T>(re, im);
}

// ---------------------------------------------------------------------------
// restriction / prolongation, fine level.  RB right-hand sides per thread:
// each column of P is loaded once and applied to all of them.  Fine fields
// of the batch are fstride apart, coarse fields cstride apart.
// ---------------------------------------------------------------------------
// the fine fields in spinor storage V (ins: their site scales for FP16)
template <typename T, typename S, int RB, typename V = C<T>>
__global__ void __launch_bounds__(256) k_restrict_fine(const int* __restrict__ members, int nbpa, int N, long long fstride,
                                const S* __restrict__ P, const V* __restrict__ in, const float* __restrict__ ins,
                                C<T>* __restrict__ out, long long cstride) {
  extern __shared__ unsigned char smem_raw[];
  T* red = reinterpret_cast<T*>(smem_raw);
  const int A = blockIdx.x, t = threadIdx.x;
  const int blk = members[A * nbpa + (t >> 4)], loc = t & 15;
  const long long sstride = fstride / 12;
  in += (long long)blockIdx.y * RB * fstride;
  if constexpr (std::is_same<V, __half2>::value) ins += (long long)blockIdx.y * RB * sstride;
  out += (long long)blockIdx.y * RB * cstride;
  C<T> v[RB][12];
#pragma unroll
  for (int r = 0; r < RB; ++r)
    load_site<T, V>(in + r * fstride, std::is_same<V, __half2>::value ? ins + r * sstride : nullptr, blk, loc, v[r]);
  for (int k = 0; k < N; ++k) {
    C<T> w[12];
    load_spinor<T, S>(P + k * fstride, blk, loc, w);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      C<T> s0 = czero<T>(), s1 = czero<T>();
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        cjfma(s0, w[c], v[r][c]);
        cjfma(s1, w[6 + c], v[r][6 + c]);
      }
      stash4<T>(red, RB * N, r * N + k, s0.x, s0.y, s1.x, s1.y);
    }
  }
  __syncthreads();
  for (int e = t; e < RB * 2 * N; e += blockDim.x) {
    const int r = e / (2 * N), q = e % (2 * N);
    out[r * cstride + (long long)A * 2 * N + q] = collect<T>(red, RB * N, q / N, r * N + q % N);
  }
}

// ---------------------------------------------------------------------------
// Restriction and prolongation of a batch on the matrix cores (FP32
// arithmetic, 8..16 fields per launch chunk, N <= 32).  Per aggregate and
// chirality half the restriction is the complex GEMM
//   out (nb x N) = V^T (nb x 96 per block, summed over the blocks) conj(P),
// the prolongation out (96 x nb per block) = P (96 x N) c (N x nb).  One
// workgroup per aggregate stages a 2^4 block of every field (and of every
// P_k for the restriction) in LDS at a time with contiguous loads, decoded
// to FP32 (FP16 fields times their site scales, FP16 P widened), and feeds
// 16x16x4 FP32 MFMA tiles from there: four real products per complex step.
// Operand layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; result register v of lane l is D[4 (l / 16) + v][l % 16].
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int TMF_NB = 16;     // fields per launch chunk
constexpr int TMF_PAD = 196;   // LDS row stride (complex) of a staged block

__device__ inline f32x4 mfma4(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <typename S, typename V>
__global__ void __launch_bounds__(256) k_restrict_fine_mfma(const int* __restrict__ members, int nbpa, int N,
                                                             long long fstride, const S* __restrict__ P,
                                                             const V* __restrict__ in, const float* __restrict__ ins,
                                                             float2* __restrict__ out, long long cstride, int nb) {
  constexpr bool HS = std::is_same<V, __half2>::value;
  __shared__ float2 vl[TMF_NB][TMF_PAD];
  __shared__ float2 pl[32][TMF_PAD];
  const int A = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int r0 = blockIdx.y * TMF_NB, nr = min(TMF_NB, nb - r0);
  const long long sstride = fstride / 12;
  const int sg = w & 1, kt = w >> 1, rr = lane & 15, kk = lane >> 4;
  f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
  constexpr int NVE = TMF_NB * 192 / 256, NPE = 32 * 192 / 256;   // staged elements per thread
  for (int bi = 0; bi < nbpa; ++bi) {
    const int blk = members[A * nbpa + bi];
    // every load of the block first, then the LDS stores (a load consumed
    // at once would stall each of them in turn)
    V va[NVE];
    float vm[NVE];
    S pa[NPE];
#pragma unroll
    for (int i = 0; i < NVE; ++i) {
      const int e = t + 256 * i, r = e / 192, q = e - r * 192;
      va[i] = szero<V>();
      vm[i] = 1.f;
      if (r < nr) {
        va[i] = in[(long long)(r0 + r) * fstride + (long long)blk * 192 + q];
        if constexpr (HS) vm[i] = ins[(long long)(r0 + r) * sstride + (long long)blk * 16 + (q & 15)];
      }
    }
#pragma unroll
    for (int i = 0; i < NPE; ++i) {
      const int e = t + 256 * i, k = e / 192, q = e - k * 192;
      pa[i] = k < N ? P[(long long)k * fstride + (long long)blk * 192 + q] : szero<S>();
    }
#pragma unroll
    for (int i = 0; i < NVE; ++i) {
      const int e = t + 256 * i, r = e / 192, q = e - r * 192;
      float2 v = ldc<float, V>(va[i]);
      v.x *= vm[i];
      v.y *= vm[i];
      vl[r][q] = v;
    }
#pragma unroll
    for (int i = 0; i < NPE; ++i) {
      const int e = t + 256 * i, k = e / 192, q = e - k * 192;
      pl[k][q] = ldc<float, S>(pa[i]);
    }
    __syncthreads();
    // the 96 components of chirality half sg: 6 spin-colour rows x 16 sites,
    // summed per block and then over the blocks (shorter chains of FP32
    // additions than one running sum over the aggregate)
    f32x4 br = {0.f, 0.f, 0.f, 0.f}, bi_ = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int s4 = 0; s4 < 96; s4 += 4) {
      const int q = sg * 96 + s4 + kk;
      const float2 a = vl[rr][q];
      const float2 b = pl[kt * 16 + rr][q];
      // conj(P) v: re = vr pr + vi pi, im = vi pr - vr pi
      br = mfma4(a.x, b.x, br);
      br = mfma4(a.y, b.y, br);
      bi_ = mfma4(a.y, b.x, bi_);
      bi_ = mfma4(-a.x, b.y, bi_);
    }
    cr += br;
    ci += bi_;
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * kk + v, k = kt * 16 + rr;
    if (r < nr && k < N) out[(long long)(r0 + r) * cstride + (long long)A * 2 * N + sg * N + k] = make_float2(cr[v], ci[v]);
  }
}

template <typename S, typename V>
__global__ void __launch_bounds__(256) k_prolong_fine_mfma(const int* __restrict__ members, int nbpa, int N,
                                                            long long fstride, const S* __restrict__ P,
                                                            const float2* __restrict__ in, V* __restrict__ out,
                                                            float* __restrict__ outs, long long cstride, int nb) {
  constexpr bool HS = std::is_same<V, __half2>::value;
  __shared__ float2 cl[TMF_NB][65];
  __shared__ float2 ol[TMF_NB][TMF_PAD];
  const int A = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int r0 = blockIdx.y * TMF_NB, nr = min(TMF_NB, nb - r0);
  const long long sstride = fstride / 12;
  const int rl = lane & 15, kk = lane >> 4;
  for (int e = t; e < TMF_NB * 2 * N; e += 256) {
    const int r = e / (2 * N), q = e - r * 2 * N;
    cl[r][q] = r < nr ? in[(long long)(r0 + r) * cstride + (long long)A * 2 * N + q] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int bi = 0; bi < nbpa; ++bi) {
    const int blk = members[A * nbpa + bi];
    // twelve 16-site row tiles (one per spin-colour component), three per wavefront
    for (int c = w; c < 12; c += 4) {
      const int sg = c / 6;
      f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
      // the tile's P entries for every k step, loaded before the products
      S pa[8];
#pragma unroll
      for (int st = 0; st < 8; ++st) {
        const int k = 4 * st + kk;
        pa[st] = k < N ? P[(long long)k * fstride + (long long)blk * 192 + c * 16 + rl] : szero<S>();
      }
#pragma unroll
      for (int st = 0; st < 8; ++st) {
        const int k0 = 4 * st;
        if (k0 >= N) break;
        const int k = k0 + kk;
        const float2 a = ldc<float, S>(pa[st]);
        const float2 b = k < N ? cl[rl][sg * N + k] : make_float2(0.f, 0.f);
        // P c: re = pr cr - pi ci, im = pr ci + pi cr
        cr = mfma4(a.x, b.x, cr);
        cr = mfma4(-a.y, b.y, cr);
        ci = mfma4(a.x, b.y, ci);
        ci = mfma4(a.y, b.x, ci);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) ol[rl][c * 16 + 4 * kk + v] = make_float2(cr[v], ci[v]);
    }
    __syncthreads();
    // one thread per (field, site) of the block writes the site
    const int r = t >> 4, loc = t & 15;
    if (r < nr) {
      float2 v[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = ol[r][c * 16 + loc];
      V* o = out + (long long)(r0 + r) * fstride;
      if constexpr (!HS) {
        float2 old[12];
        load_spinor<float, V>(o, blk, loc, old);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = cadd(v[c], old[c]);
      }
      store_site<float, V>(o, HS ? outs + (long long)(r0 + r) * sstride : nullptr, blk, loc, v);
    }
    __syncthreads();
  }
}

// whether the matrix-core transfer takes a batch of nb with N test vectors
inline bool use_transfer_mfma(int nb, int N, int asz) { return nb >= 8 && N <= 32 && asz <= 1024; }

template <typename S, typename V>
void restrict_fine_mfma(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const S* P, const V* in,
                        const float* ins, float2* out, hipStream_t s, int nb) {
  const long long fs = (long long)g.nblk * 192, cs = (long long)a.nagg * 2 * N;
  k_restrict_fine_mfma<S, V><<<dim3(a.nagg, (nb + TMF_NB - 1) / TMF_NB), 256, 0, s>>>(ad.members, a.asz / 16, N, fs,
                                                                                     P, in, ins, out, cs, nb);
  DD_LAUNCH_CHECK();
}

template <typename S, typename V>
void prolong_fine_mfma(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const S* P, const float2* in,
                       V* out, float* outs, hipStream_t s, int nb) {
  const long long fs = (long long)g.nblk * 192, cs = (long long)a.nagg * 2 * N;
  k_prolong_fine_mfma<S, V><<<dim3(a.nagg, (nb + TMF_NB - 1) / TMF_NB), 256, 0, s>>>(ad.members, a.asz / 16, N, fs,
                                                                                    P, in, out, outs, cs, nb);
  DD_LAUNCH_CHECK();
}

template <typename T, typename S>
void restrict_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const S* P,
                   const C<T>* in, C<T>* out, hipStream_t s, int nb) {
  if constexpr (std::is_same<T, float>::value) {
    if (use_transfer_mfma(nb, N, a.asz)) return restrict_fine_mfma<S, float2>(g, a, ad, N, P, in, nullptr, out, s, nb);
  }
  const long long fs = (long long)g.nblk * 192, cs = (long long)a.nagg * 2 * N;
  rhs_chunks<T>(nb, [&](auto rb, int first, int nch) {
    constexpr int RB = decltype(rb)::value;
    const size_t sm = (size_t)((a.asz + 63) / 64) * RB * N * 4 * sizeof(T);
    k_restrict_fine<T, S, RB><<<dim3(a.nagg, nch), a.asz, sm, s>>>(ad.members, a.asz / 16, N, fs, P,
                                                                   in + first * fs, nullptr, out + first * cs, cs);
  });
  DD_LAUNCH_CHECK();
}

void restrict_fine_hs(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const __half2* P,
                      const __half2* in, const float* ins, float2* out, hipStream_t s, int nb) {
  if (use_transfer_mfma(nb, N, a.asz)) return restrict_fine_mfma<__half2, __half2>(g, a, ad, N, P, in, ins, out, s, nb);
  const long long fs = (long long)g.nblk * 192, cs = (long long)a.nagg * 2 * N, ss = (long long)g.nblk * 16;
  rhs_chunks<float>(nb, [&](auto rb, int first, int nch) {
    constexpr int RB = decltype(rb)::value;
    const size_t sm = (size_t)((a.asz + 63) / 64) * RB * N * 4 * sizeof(float);
    k_restrict_fine<float, __half2, RB, __half2><<<dim3(a.nagg, nch), a.asz, sm, s>>>(
        ad.members, a.asz / 16, N, fs, P, in + first * fs, ins + first * ss, out + first * cs, cs);
  });
  DD_LAUNCH_CHECK();
}

// out += P in for V = C<T>; out = P in, encoded with new site scales
// (outs), for FP16 spinors
template <typename T, typename S, int RB, typename V = C<T>>
__global__ void __launch_bounds__(256) k_prolong_fine(const int* __restrict__ blk_agg, int nblk, int N, long long fstride,
                               const S* __restrict__ P, const C<T>* __restrict__ in,
                               V* __restrict__ out, float* __restrict__ outs, long long cstride) {
  constexpr bool HS = std::is_same<V, __half2>::value;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15;
  if (blk >= nblk) return;
  const long long sstride = fstride / 12;
  in += (long long)blockIdx.y * RB * cstride;
  out += (long long)blockIdx.y * RB * fstride;
  if constexpr (HS) outs += (long long)blockIdx.y * RB * sstride;
  const int A = blk_agg[blk];
  C<T> acc[RB][12];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if constexpr (HS) {
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[r][c] = czero<T>();
    } else {
      load_spinor<T>(out + r * fstride, blk, loc, acc[r]);
    }
  }
  for (int k = 0; k < N; ++k) {
    C<T> w[12];
    load_spinor<T, S>(P + k * fstride, blk, loc, w);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const C<T>* phi = in + r * cstride + (long long)A * 2 * N;
      const C<T> p0 = phi[k], p1 = phi[N + k];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        cfma(acc[r][c], w[c], p0);
        cfma(acc[r][6 + c], w[6 + c], p1);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) store_site<T, V>(out + r * fstride, HS ? outs + r * sstride : nullptr, blk, loc, acc[r]);
}

template <typename T, typename S>
void prolong_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const S* P,
                  const C<T>* in, C<T>* out, hipStream_t s, int nb) {
  if constexpr (std::is_same<T, float>::value) {
    if (use_transfer_mfma(nb, N, a.asz)) return prolong_fine_mfma<S, float2>(g, a, ad, N, P, in, out, nullptr, s, nb);
  }
  const long long fs = (long long)g.nblk * 192, cs = (long long)a.nagg * 2 * N;
  rhs_chunks<T>(nb, [&](auto rb, int first, int nch) {
    constexpr int RB = decltype(rb)::value;
    k_prolong_fine<T, S, RB><<<dim3(nblocks((size_t)g.nblk * 16, 256), nch), 256, 0, s>>>(
        ad.member_agg, g.nblk, N, fs, P, in + first * cs, out + first * fs, nullptr, cs);
  });
  DD_LAUNCH_CHECK();
}

void prolong_fine_hs(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const __half2* P,
                     const float2* in, __half2* out, float* outs, hipStream_t s, int nb) {
  if (use_transfer_mfma(nb, N, a.asz)) return prolong_fine_mfma<__half2, __half2>(g, a, ad, N, P, in, out, outs, s, nb);
  const long long fs = (long long)g.nblk * 192, cs = (long long)a.nagg * 2 * N, ss = (long long)g.nblk * 16;
  rhs_chunks<float>(nb, [&](auto rb, int first, int nch) {
    constexpr int RB = decltype(rb)::value;
    k_prolong_fine<float, __half2, RB, __half2><<<dim3(nblocks((size_t)g.nblk * 16, 256), nch), 256, 0, s>>>(
        ad.member_agg, g.nblk, N, fs, P, in + first * cs, out + first * fs, outs + first * ss, cs);
  });
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// restriction / prolongation, coarse level (d components per site)
// ---------------------------------------------------------------------------
template <typename T, typename S, int RB>
__global__ void k_restrict_coarse(const int* __restrict__ members, int asz, int d, int N,
                                  long long fstride, const S* __restrict__ P,
                                  const C<T>* __restrict__ in, C<T>* __restrict__ out, long long cstride) {
  extern __shared__ unsigned char smem_raw[];
  T* red = reinterpret_cast<T*>(smem_raw);
  const int A = blockIdx.x, t = threadIdx.x;
  in += (long long)blockIdx.y * RB * fstride;
  out += (long long)blockIdx.y * RB * cstride;
  const bool valid = t < asz * d;
  const int sl = valid ? t / d : 0, i = valid ? t % d : 0;
  const int site = members[A * asz + sl];
  const long long e = (long long)site * d + i;
  C<T> v[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) v[r] = valid ? in[r * fstride + e] : czero<T>();
  const bool up = i < d / 2;
  for (int k = 0; k < N; ++k) {
    const C<T> pk = valid ? ldc<T, S>(P[k * fstride + e]) : czero<T>();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      C<T> p = czero<T>();
      cjfma(p, pk, v[r]);
      stash4<T>(red, RB * N, r * N + k, up ? p.x : T(0), up ? p.y : T(0), up ? T(0) : p.x,
                up ? T(0) : p.y);
    }
  }
  __syncthreads();
  for (int q2 = t; q2 < RB * 2 * N; q2 += blockDim.x) {
    const int r = q2 / (2 * N), q = q2 % (2 * N);
    out[r * cstride + (long long)A * 2 * N + q] = collect<T>(red, RB * N, q / N, r * N + q % N);
  }
}

template <typename T, typename S>
void restrict_coarse(const AggTables& a, const AggDev& ad, int d, int N, long long V,
                     const S* P, const C<T>* in, C<T>* out, hipStream_t s, int nb) {
  const int rows = a.asz * d;
  DD_REQUIRE(rows <= 1024, "coarse aggregate too large for one workgroup");
  const int wg = 64 * ((rows + 63) / 64);
  const long long fs = V * d, cs = (long long)a.nagg * 2 * N;
  rhs_chunks<T>(nb, [&](auto rb, int first, int nch) {
    constexpr int RB = decltype(rb)::value;
    const size_t sm = (size_t)(wg / 64) * RB * N * 4 * sizeof(T);
    k_restrict_coarse<T, S, RB><<<dim3(a.nagg, nch), wg, sm, s>>>(ad.members, a.asz, d, N, fs, P,
                                                                  in + first * fs, out + first * cs, cs);
  });
  DD_LAUNCH_CHECK();
}

template <typename T, typename S, int RB>
__global__ void k_prolong_coarse(const int* __restrict__ site_agg, long long V, int d, int N,
                                 long long fstride, const S* __restrict__ P,
                                 const C<T>* __restrict__ in, C<T>* __restrict__ out, long long cstride) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= V * d) return;
  in += (long long)blockIdx.y * RB * cstride;
  out += (long long)blockIdx.y * RB * fstride;
  const int site = (int)(e / d), i = (int)(e % d);
  const int sigma = i < d / 2 ? 0 : 1;
  const long long po = (long long)site_agg[site] * 2 * N + sigma * N;
  C<T> acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = out[r * fstride + e];
  for (int k = 0; k < N; ++k) {
    const C<T> pk = ldc<T, S>(P[k * fstride + e]);
#pragma unroll
    for (int r = 0; r < RB; ++r) cfma(acc[r], pk, in[r * cstride + po + k]);
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) out[r * fstride + e] = acc[r];
}

template <typename T, typename S>
void prolong_coarse(const AggTables& a, const AggDev& ad, int d, int N, long long V, const S* P,
                    const C<T>* in, C<T>* out, hipStream_t s, int nb) {
  const long long fs = V * d, cs = (long long)a.nagg * 2 * N;
  rhs_chunks<T>(nb, [&](auto rb, int first, int nch) {
    constexpr int RB = decltype(rb)::value;
    k_prolong_coarse<T, S, RB><<<dim3(nblocks((size_t)V * d, 256), nch), 256, 0, s>>>(
        ad.member_agg, V, d, N, fs, P, in + first * cs, out + first * fs, cs);
  });
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Block orthonormalisation (FP64).  One workgroup per (aggregate, chirality);
// every thread owns the same element positions in all N fields, so a thread
// only re-reads what it wrote itself.  Gram-Schmidt with one full
// re-orthogonalisation pass, in index order.
// ---------------------------------------------------------------------------
constexpr int NMAX = 32;   // max test vectors per level
constexpr int EPT = 8;     // max elements per thread

// Element e of the restriction of a field to (aggregate A, chirality sigma):
// the order is free (the result does not depend on it) and is chosen so that
// consecutive elements are consecutive in memory.
struct FineMap {
  const int* members;
  int nbpa;
  __device__ long long operator()(int A, int sigma, int e) const {
    const int asz = nbpa * 16;
    const int c = 6 * sigma + e / asz, ts = e % asz;
    const int blk = members[A * nbpa + (ts >> 4)];
    return ((long long)blk * 12 + c) * 16 + (ts & 15);
  }
};
struct CoarseMap {
  const int* members;
  int asz, d;
  __device__ long long operator()(int A, int sigma, int e) const {
    const int h = d / 2;
    const int sl = e / h, c = sigma * h + e % h;
    return (long long)members[A * asz + sl] * d + c;
  }
};

// Orthonormalisation of the N test vectors restricted to (aggregate,
// chirality): one workgroup per pair, Cholesky QR applied twice.  A pass
// forms the Gram matrix G = V^H V (chunks of the vectors staged in LDS,
// one upper-triangle entry per thread), factors G = R^H R (R upper
// triangular, positive diagonal), and writes V R^-1.  The Q factor with
// positive diagonal R is unique, so this is the Gram-Schmidt result of the
// paper's construction up to rounding; the second pass restores
// orthogonality to working precision.  A vector that depends on the
// earlier ones (zero pivot) gives a zero column, as Gram-Schmidt does.
constexpr int ORTH_CHUNK = 16;    // elements per LDS chunk of the Gram pass
constexpr int ORTH_APPLY = 64;    // elements per LDS chunk of the V R^-1 pass

__device__ inline void orth_pair(int p, int N, int& i, int& j) {
  // p -> (i, j), i <= j, row by row of the upper triangle
  i = 0;
  int row = N;
  while (p >= row) {
    p -= row;
    --row;
    ++i;
  }
  j = i + p;
}

template <class Map>
__global__ void __launch_bounds__(256) k_orth(Map map, int m, int N, long long fstride,
                                              const double2* __restrict__ tv, double2* __restrict__ P,
                                              int* __restrict__ flag) {
  __shared__ double2 chunk[NMAX * ORTH_APPLY];
  __shared__ double2 R[NMAX * NMAX];   // Gram matrix, then R (upper triangle)
  __shared__ double2 X[NMAX * NMAX];   // R^-1 (upper triangle)
  __shared__ int dep[NMAX];
  const int A = blockIdx.x >> 1, sigma = blockIdx.x & 1;
  const int t = threadIdx.x;
  const int npairs = N * (N + 1) / 2;
  constexpr int PPT = (NMAX * (NMAX + 1) / 2 + 255) / 256;
  for (int pass = 0; pass < 2; ++pass) {
    const double2* src = pass == 0 ? tv : P;
    // Gram matrix
    double2 acc[PPT];
    int pi[PPT], pj[PPT];
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      acc[r] = czero<double>();
      pi[r] = pj[r] = 0;
      if (t + 256 * r < npairs) orth_pair(t + 256 * r, N, pi[r], pj[r]);
    }
    for (int e0 = 0; e0 < m; e0 += ORTH_CHUNK) {
      for (int idx = t; idx < N * ORTH_CHUNK; idx += 256) {
        const int j = idx / ORTH_CHUNK, e = e0 + idx % ORTH_CHUNK;
        chunk[idx] = e < m ? src[j * fstride + map(A, sigma, e)] : czero<double>();
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < PPT; ++r)
        if (t + 256 * r < npairs) {
          const double2* a = chunk + pi[r] * ORTH_CHUNK;
          const double2* b = chunk + pj[r] * ORTH_CHUNK;
#pragma unroll
          for (int q = 0; q < ORTH_CHUNK; ++q) cjfma(acc[r], a[q], b[q]);
        }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < PPT; ++r)
      if (t + 256 * r < npairs) R[pi[r] * NMAX + pj[r]] = acc[r];
    __syncthreads();
    // Cholesky G = R^H R in place (upper triangle): thread j < N owns
    // column j; step k fixes row k
    for (int k = 0; k < N; ++k) {
      if (t == k) {
        double dk = R[k * NMAX + k].x;
        for (int i = 0; i < k; ++i) {
          const double2 r = R[i * NMAX + k];
          dk -= r.x * r.x + r.y * r.y;
        }
        const double gkk = R[k * NMAX + k].x;
        // a column whose part orthogonal to the earlier ones is below the
        // rounding level of the Gram matrix (relative 1e-12) cannot be
        // orthonormalised accurately from it: reported to the host
        if (!(dk > 1e-12 * gkk)) *flag = 1;
        const bool zero = !(gkk > 0.0) || !(dk > 1e-28 * gkk);
        dep[k] = zero ? 1 : 0;
        R[k * NMAX + k] = make_double2(zero ? 0.0 : sqrt(dk), 0.0);
      }
      __syncthreads();
      if (t > k && t < N) {
        double2 g = R[k * NMAX + t];
        for (int i = 0; i < k; ++i) g = csub(g, cjmul(R[i * NMAX + k], R[i * NMAX + t]));
        const double rkk = R[k * NMAX + k].x;
        R[k * NMAX + t] = rkk > 0.0 ? cscale(g, 1.0 / rkk) : czero<double>();
      }
      __syncthreads();
    }
    // X = R^-1: thread j < N solves column j (zero rows and columns for
    // dependent vectors)
    if (t < N) {
      const int j = t;
      for (int i = 0; i < N; ++i) X[i * NMAX + j] = czero<double>();
      if (!dep[j]) {
        X[j * NMAX + j] = make_double2(1.0 / R[j * NMAX + j].x, 0.0);
        for (int i = j - 1; i >= 0; --i) {
          if (dep[i]) continue;
          double2 sacc = czero<double>();
          for (int k = i + 1; k <= j; ++k) cfma(sacc, R[i * NMAX + k], X[k * NMAX + j]);
          X[i * NMAX + j] = cscale(sacc, -1.0 / R[i * NMAX + i].x);
        }
      }
    }
    __syncthreads();
    // P = V X, chunks of ORTH_APPLY elements staged in LDS (the whole
    // chunk is read before any of it is written, so the second pass may
    // work in place); thread t forms outputs (element, column) t, t+256, ...
    for (int e0 = 0; e0 < m; e0 += ORTH_APPLY) {
      for (int idx = t; idx < N * ORTH_APPLY; idx += 256) {
        const int j = idx / ORTH_APPLY, e = e0 + idx % ORTH_APPLY;
        chunk[idx] = e < m ? src[j * fstride + map(A, sigma, e)] : czero<double>();
      }
      __syncthreads();
      for (int idx = t; idx < N * ORTH_APPLY; idx += 256) {
        const int j = idx / ORTH_APPLY, q = idx % ORTH_APPLY, e = e0 + q;
        if (e >= m) continue;
        double2 o = czero<double>();
        for (int i = 0; i <= j; ++i) cfma(o, chunk[i * ORTH_APPLY + q], X[i * NMAX + j]);
        P[j * fstride + map(A, sigma, e)] = o;
      }
      __syncthreads();
    }
  }
}

void orthonormalise_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N,
                         const double2* tv, double2* P, int* flag, hipStream_t s) {
  const int m = a.asz * 6;
  DD_REQUIRE(N <= NMAX, "too many test vectors");
  DD_REQUIRE(N <= m, "more test vectors than the aggregate dimension");
  DD_REQUIRE(m <= 256 * EPT, "aggregate too large");
  k_orth<FineMap><<<2 * a.nagg, 256, 0, s>>>(FineMap{ad.members, a.asz / 16}, m, N,
                                            (long long)g.nblk * 192, tv, P, flag);
  DD_LAUNCH_CHECK();
}

void orthonormalise_coarse(const AggTables& a, const AggDev& ad, int d, int N, long long V,
                           const double2* tv, double2* P, int* flag, hipStream_t s) {
  const int m = a.asz * (d / 2);
  DD_REQUIRE(N <= NMAX, "too many test vectors");
  DD_REQUIRE(N <= m, "more test vectors than the aggregate dimension");
  DD_REQUIRE(m <= 256 * EPT, "aggregate too large");
  k_orth<CoarseMap><<<2 * a.nagg, 256, 0, s>>>(CoarseMap{ad.members, a.asz, d}, m, N, V * d, tv, P, flag);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Galerkin, fine level: grid (aggregate, coarse column (sigma, k)), one
// thread per fine site of the aggregate.  For the column u = P_k restricted
// to chirality sigma the thread forms, in turn, the self part
//   y = A(x) u(x) - 1/2 sum of the hops whose both ends lie in the aggregate
// and the four forward face parts y = -1/2 (1-g_mu) U_mu(x) u(x+mu) (x+mu
// outside), and projects each on the rows P_k'(x) (both chiralities).
// ---------------------------------------------------------------------------
struct GalFineGeom {
  int nb[4];
  int agg[4];
};

// Galerkin grids: workgroup bid of 8 * ceil(nagg / 8) * ncol handles
// (aggregate A, column col) such that the ncol columns of an aggregate run
// one after another on one XCD (workgroup i is dispatched to XCD i mod 8),
// whose L2 then serves the aggregate's links, clover and rows of P to all
// of them.  Returns false for the padding workgroups.
__device__ inline bool agg_col_xcd(int bid, int nagg, int ncol, int& A, int& col) {
  const int apx = (nagg + 7) / 8;
  const int j = bid >> 3;
  A = (bid & 7) * apx + j / ncol;
  col = j % ncol;
  return A < nagg;
}
inline unsigned agg_col_grid(int nagg, int ncol) { return 8u * (unsigned)((nagg + 7) / 8) * (unsigned)ncol; }

// y += -1/2 * hop of the column restricted to chirality SIGMA: the other
// spinor half is a compile-time zero (not loaded), and the factor -1/2 is
// applied to the input so that the hop accumulates straight into y
template <int MU, bool FWD, int SIGMA>
__device__ inline void gal_hop(const FineOpView<double>& op, const double2* __restrict__ Pk, int blk, int loc,
                               double2 y[12]) {
  constexpr int bit = 1 << MU;
  int nb;
  if constexpr (FWD) nb = (loc & bit) ? op.nbr[blk * 8 + 2 * MU] : blk;
  else nb = (loc & bit) ? blk : op.nbr[blk * 8 + 2 * MU + 1];
  double2 psi[12], u[9];
  const double2* p = Pk + (long long)nb * 192 + (loc ^ bit);
#pragma unroll
  for (int c = 0; c < 12; ++c)
    psi[c] = (c / 6) == SIGMA ? cscale(p[c * 16], -0.5) : czero<double>();
  if constexpr (FWD) load_link<double>(op.U, blk, loc, MU, u);
  else load_link<double>(op.U, nb, loc ^ bit, MU, u);
  hop_apply<double, MU, FWD>(psi, u, y);
}

template <int MU, int SIGMA>
__device__ inline void gal_hops_inside(const FineOpView<double>& op, const double2* Pk, int blk, int loc,
                                       const bool* fin, const bool* bin, double2 y[12]) {
  if (fin[MU]) gal_hop<MU, true, SIGMA>(op, Pk, blk, loc, y);
  if (bin[MU]) gal_hop<MU, false, SIGMA>(op, Pk, blk, loc, y);
}

// part tau of the column (SIGMA, k) at this thread's site: tau = 0 the self
// part (clover and the hops inside the aggregate), tau = 1 + mu the forward
// face part across the +mu face
template <int SIGMA>
__device__ inline void gal_part(const FineOpView<double>& op, const double2* __restrict__ Pk, int blk, int loc,
                                const bool* fin, const bool* bin, int tau, double2 y[12]) {
  if (tau == 0) {
    // the clover is block diagonal in chirality: only block SIGMA acts
    double2 u[6];
    const double2* p = Pk + (long long)blk * 192 + loc + 6 * SIGMA * 16;
#pragma unroll
    for (int c = 0; c < 6; ++c) u[c] = p[c * 16];
#pragma unroll
    for (int c = 0; c < 6; ++c) y[6 * (1 - SIGMA) + c] = czero<double>();
    const double2* a = op.A + (long long)blk * 576 + loc;
    clover_block<double>(SIGMA, [&](int e) { return a[e * 16]; }, u, y + 6 * SIGMA);
    gal_hops_inside<0, SIGMA>(op, Pk, blk, loc, fin, bin, y);
    gal_hops_inside<1, SIGMA>(op, Pk, blk, loc, fin, bin, y);
    gal_hops_inside<2, SIGMA>(op, Pk, blk, loc, fin, bin, y);
    gal_hops_inside<3, SIGMA>(op, Pk, blk, loc, fin, bin, y);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) y[c] = czero<double>();
    const int mu = tau - 1;
    if (!fin[mu]) {
      if (mu == 0) gal_hop<0, true, SIGMA>(op, Pk, blk, loc, y);
      else if (mu == 1) gal_hop<1, true, SIGMA>(op, Pk, blk, loc, y);
      else if (mu == 2) gal_hop<2, true, SIGMA>(op, Pk, blk, loc, y);
      else gal_hop<3, true, SIGMA>(op, Pk, blk, loc, y);
    }
  }
}

__global__ void __launch_bounds__(256) k_galerkin_fine(GalFineGeom gg, const int* __restrict__ members,
                                                       int nbpa, int N, int nagg, FineOpView<double> op,
                                                       const double2* __restrict__ P, long long fstride,
                                                       double2* __restrict__ Dc) {
  __shared__ double red[4 * NMAX * 4];
  int A, col;
  if (!agg_col_xcd(blockIdx.x, nagg, 2 * N, A, col)) return;
  const int sigma = col / N, k = col % N;
  const int t = threadIdx.x;
  const int blk = members[A * nbpa + (t >> 4)], loc = t & 15;
  // fine coordinates -> which hops stay inside the aggregate
  bool fin[4], bin[4];
  {
    int bcs[4];
    block_decode(gg.nb, blk, bcs);
    for (int mu = 0; mu < 4; ++mu) {
      const int bc = bcs[mu];
      const int x = 2 * bc + ((loc >> mu) & 1);
      const int xm = x % gg.agg[mu];
      fin[mu] = xm != gg.agg[mu] - 1;
      bin[mu] = xm != 0;
    }
  }
  const double2* Pk = P + k * fstride;
  const int twoN = 2 * N;
#pragma unroll 1
  for (int tau = 0; tau < 5; ++tau) {
    double2 y[12];
    if (sigma == 0) gal_part<0>(op, Pk, blk, loc, fin, bin, tau, y);
    else gal_part<1>(op, Pk, blk, loc, fin, bin, tau, y);
    // a face part is nonzero only on the aggregate's face sites: the other
    // threads skip the loads of the rows of P and contribute zeros
    const bool live = tau == 0 || !fin[tau - 1];
#pragma unroll 2
    for (int kp = 0; kp < N; ++kp) {
      double2 p0 = czero<double>(), p1 = czero<double>();
      if (live) {
        double2 w[12];
        load_spinor<double>(P + kp * fstride, blk, loc, w);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          cjfma(p0, w[c], y[c]);
          cjfma(p1, w[6 + c], y[6 + c]);
        }
      }
      stash4<double>(red, N, kp, p0.x, p0.y, p1.x, p1.y);
    }
    __syncthreads();
    if (t < twoN)
      Dc[(((long long)A * 5 + tau) * twoN + t) * twoN + col] = collect<double>(red, N, t / N, t % N);
    __syncthreads();
  }
}

void galerkin_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N,
                   const FineOpView<double>& op, const double2* P, double2* Dc, hipStream_t s) {
  DD_REQUIRE(a.asz == 256, "fine Galerkin kernel expects 4^4-site aggregates");
  DD_REQUIRE(N <= NMAX, "too many test vectors");
  GalFineGeom gg;
  for (int mu = 0; mu < 4; ++mu) { gg.nb[mu] = g.nb[mu]; gg.agg[mu] = a.agg[mu]; }
  k_galerkin_fine<<<agg_col_grid(a.nagg, 2 * N), 256, 0, s>>>(gg, ad.members, a.asz / 16, N, a.nagg, op, P,
                                                              (long long)g.nblk * 192, Dc);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Galerkin, coarse level: grid (aggregate, group of columns), one thread
// per (site of the aggregate, row i of level l).
// ---------------------------------------------------------------------------
struct GalCoarseGeom {
  int dims[4];
  int agg[4];
};


// KG consecutive columns (same chirality half) per workgroup: each operator
// entry loaded is applied to all of them (KG = 4 where the level has
// aggregates enough to keep the device busy with a quarter of the
// workgroups, else 1)

// row i of a column-major block times the KG columns' vectors at site nb,
// restricted to the components [j0, j1)
template <int KG>
__device__ inline void colmajor_row_kg(const double2* M, const double2* P, long long fstride, long long nb,
                                       int k0, int nk, int i, int d, int j0, int j1, double2 (&y)[KG]) {
  for (int j = j0; j < j1; ++j) {
    const double2 m = M[(size_t)j * d + i];
#pragma unroll
    for (int g = 0; g < KG; ++g)
      if (g < nk) cfma(y[g], m, P[(k0 + g) * fstride + nb * d + j]);
  }
}

template <int GAL_KG>
__global__ void k_galerkin_coarse(GalCoarseGeom gg, const int* __restrict__ members, int asz, int N, int nagg,
                                  CoarseOpView<double> op, const double2* __restrict__ P,
                                  long long fstride, double2* __restrict__ Dc) {
  extern __shared__ unsigned char smem_raw[];
  double* red = reinterpret_cast<double*>(smem_raw);
  const int d = op.d, h = d / 2;
  const int ngs = (N + GAL_KG - 1) / GAL_KG;   // column groups per chirality
  int A, grp;
  if (!agg_col_xcd(blockIdx.x, nagg, 2 * ngs, A, grp)) return;
  const int sigma = grp / ngs, k0 = (grp % ngs) * GAL_KG;
  const int nk = min(GAL_KG, N - k0);
  const int j0 = sigma * h, j1 = j0 + h;
  const int t = threadIdx.x;
  const bool valid = t < asz * d;
  const int sl = valid ? t / d : 0, i = valid ? t % d : 0;
  const int site = members[A * asz + sl];
  bool fin[4], bin[4];
  {
    int r = site;
    for (int mu = 0; mu < 4; ++mu) {
      const int x = r % gg.dims[mu];
      r /= gg.dims[mu];
      const int xm = x % gg.agg[mu];
      fin[mu] = xm != gg.agg[mu] - 1;
      bin[mu] = xm != 0;
    }
  }
  const size_t bsz = (size_t)d * d;
  const double2* Kx = op.K + (size_t)site * 9 * bsz;
  const int* nb9 = op.nbr9 + (size_t)site * 9;
  const int twoN = 2 * N;
  for (int tau = 0; tau < 5; ++tau) {
    double2 y[GAL_KG];
#pragma unroll
    for (int g = 0; g < GAL_KG; ++g) y[g] = czero<double>();
    if (valid) {
      if (tau == 0) {
        colmajor_row_kg<GAL_KG>(Kx, P, fstride, site, k0, nk, i, d, j0, j1, y);
        for (int mu = 0; mu < 4; ++mu) {
          if (fin[mu]) colmajor_row_kg<GAL_KG>(Kx + (1 + mu) * bsz, P, fstride, nb9[1 + mu], k0, nk, i, d, j0, j1, y);
          if (bin[mu]) colmajor_row_kg<GAL_KG>(Kx + (5 + mu) * bsz, P, fstride, nb9[5 + mu], k0, nk, i, d, j0, j1, y);
        }
      } else {
        const int mu = tau - 1;
        if (!fin[mu]) colmajor_row_kg<GAL_KG>(Kx + (1 + mu) * bsz, P, fstride, nb9[1 + mu], k0, nk, i, d, j0, j1, y);
      }
    }
    const bool up = i < h;
    for (int g = 0; g < nk; ++g) {
      for (int kp = 0; kp < N; ++kp) {
        double2 p = czero<double>();
        if (valid) cjfma(p, P[kp * fstride + (size_t)site * d + i], y[g]);
        stash4<double>(red, N, kp, up ? p.x : 0.0, up ? p.y : 0.0, up ? 0.0 : p.x, up ? 0.0 : p.y);
      }
      __syncthreads();
      const int col = sigma * N + k0 + g;
      if (t < twoN)
        Dc[(((long long)A * 5 + tau) * twoN + t) * twoN + col] = collect<double>(red, N, t / N, t % N);
      __syncthreads();
    }
  }
}

void galerkin_coarse(const CoarseGeom& cg, const AggTables& a, const AggDev& ad, int N,
                     const CoarseOpView<double>& op, const double2* P, double2* Dc, hipStream_t s, int cols) {
  const int rows = a.asz * cg.d;
  DD_REQUIRE(rows <= 1024, "coarse aggregate too large for one workgroup");
  DD_REQUIRE(N <= NMAX, "too many test vectors");
  GalCoarseGeom gg;
  for (int mu = 0; mu < 4; ++mu) { gg.dims[mu] = cg.dims[mu]; gg.agg[mu] = a.agg[mu]; }
  const int wg = 64 * ((rows + 63) / 64);
  const size_t sm = (size_t)(wg / 64) * N * 4 * sizeof(double);
  const bool four = cols == 4 || (cols == 0 && (long long)a.nagg * 2 * ((N + 3) / 4) >= 2048);
  if (four) {
    const int ngs = (N + 3) / 4;
    k_galerkin_coarse<4><<<agg_col_grid(a.nagg, 2 * ngs), wg, sm, s>>>(gg, ad.members, a.asz, N, a.nagg, op, P,
                                                                       (long long)cg.V * cg.d, Dc);
  } else {
    k_galerkin_coarse<1><<<agg_col_grid(a.nagg, 2 * N), wg, sm, s>>>(gg, ad.members, a.asz, N, a.nagg, op, P,
                                                                     (long long)cg.V * cg.d, Dc);
  }
  DD_LAUNCH_CHECK();
}

#define DD_INST(T, S)                                                                               \
  template void restrict_fine<T, S>(const FineGeom&, const AggTables&, const AggDev&, int, const S*,  \
                                    const C<T>*, C<T>*, hipStream_t, int);                        \
  template void prolong_fine<T, S>(const FineGeom&, const AggTables&, const AggDev&, int, const S*,   \
                                   const C<T>*, C<T>*, hipStream_t, int);                         \
  template void restrict_coarse<T, S>(const AggTables&, const AggDev&, int, int, long long,         \
                                      const S*, const C<T>*, C<T>*, hipStream_t, int);            \
  template void prolong_coarse<T, S>(const AggTables&, const AggDev&, int, int, long long, const S*, \
                                     const C<T>*, C<T>*, hipStream_t, int);
DD_INST(double, double2)
DD_INST(float, float2)
DD_INST(float, __half2)
#undef DD_INST

}  // namespace ddamg
