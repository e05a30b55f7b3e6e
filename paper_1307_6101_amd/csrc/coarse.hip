// Coarse-level kernels: block-stencil apply, SAP colour pass with block MR,
// and the odd-even pieces of the coarsest solve.
#include "coarse.h"
#include "coarse_dev.h"

#include <algorithm>

namespace ddamg {

CoarseGeom make_coarse_geom(const int dims[4], int d, const int sap[4]) {
  CoarseGeom g;
  g.V = 1;
  for (int mu = 0; mu < 4; ++mu) { g.dims[mu] = dims[mu]; g.V *= dims[mu]; g.sap[mu] = sap[mu]; }
  g.d = d;
  auto idx = [&](const int c[4]) {
    return c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]));
  };
  g.nbr9.resize((size_t)g.V * 9);
  g.bipartite = true;
  for (int mu = 0; mu < 4; ++mu) g.bipartite = g.bipartite && (dims[mu] % 2 == 0);
  for (int s = 0; s < g.V; ++s) {
    int c[4], r = s;
    for (int mu = 0; mu < 4; ++mu) { c[mu] = r % dims[mu]; r /= dims[mu]; }
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[mu] = (cc[mu] + (dir == 0 ? 1 : dims[mu] - 1)) % dims[mu];
        g.nbr9[s * 9 + 1 + mu + 4 * dir] = idx(cc);
      }
    g.nbr9[s * 9] = s;
    if (((c[0] + c[1] + c[2] + c[3]) & 1) == 0) g.even.push_back(s);
    else g.odd.push_back(s);
  }
  // SAP blocks (only needed where the level is smoothed; sap[0] == 0 disables)
  g.nblk = 0;
  g.bs = 0;
  if (sap[0] > 0) {
    int nb[4];
    g.bs = 1;
    g.nblk = 1;
    for (int mu = 0; mu < 4; ++mu) {
      nb[mu] = dims[mu] / sap[mu];
      g.bs *= sap[mu];
      g.nblk *= nb[mu];
    }
    std::vector<int> order[2];
    for (int b = 0; b < g.nblk; ++b) {
      int c[4], r = b;
      for (int mu = 0; mu < 4; ++mu) { c[mu] = r % nb[mu]; r /= nb[mu]; }
      order[(c[0] + c[1] + c[2] + c[3]) & 1].push_back(b);
    }
    g.blk_sites.resize((size_t)g.nblk * g.bs);
    g.site_blk.resize(g.V);
    g.site_pos.resize(g.V);
    g.inmask.resize(g.V);
    int nbk = 0;
    for (int col = 0; col < 2; ++col)
      for (int b : order[col]) {
        int c[4], r = b;
        for (int mu = 0; mu < 4; ++mu) { c[mu] = r % nb[mu]; r /= nb[mu]; }
        for (int l = 0; l < g.bs; ++l) {
          int lc[4], rr = l;
          for (int mu = 0; mu < 4; ++mu) { lc[mu] = rr % sap[mu]; rr /= sap[mu]; }
          int sc[4];
          for (int mu = 0; mu < 4; ++mu) sc[mu] = c[mu] * sap[mu] + lc[mu];
          int site = idx(sc);
          g.blk_sites[(size_t)nbk * g.bs + l] = site;
          g.site_blk[site] = nbk;
          g.site_pos[site] = nbk * g.bs + l;
        }
        ++nbk;
      }
    // indexed by block-major position, which a site kernel knows without a
    // table read
    for (int s = 0; s < g.V; ++s) {
      unsigned m = 1u;
      for (int k = 1; k < 9; ++k)
        if (g.site_blk[g.nbr9[s * 9 + k]] == g.site_blk[s]) m |= 1u << k;
      g.inmask[g.site_pos[s]] = m;
    }
    g.kmax = 0;
    for (int s = 0; s < g.V; ++s) g.kmax = std::max(g.kmax, __builtin_popcount(g.inmask[s]));
  }
  return g;
}

// ---------------------------------------------------------------------------
// nine-block expansion (gamma5-symmetry gives the backward blocks)
// ---------------------------------------------------------------------------
template <typename S> __device__ inline S store_as(double2 v);
template <> __device__ inline double2 store_as<double2>(double2 v) { return v; }
template <> __device__ inline float2 store_as<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ inline __half2 store_as<__half2>(double2 v) {
  return __floats2half2_rn((float)v.x, (float)v.y);
}

template <typename S>
__global__ void k_expand(const double2* __restrict__ D5, const int* __restrict__ nbr9, int d,
                         S* __restrict__ K) {
  const int x = blockIdx.x, k = blockIdx.y;
  const int h = d / 2;
  const size_t bsz = (size_t)d * d;
  S* o = K + ((size_t)x * 9 + k) * bsz;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int j = e / d, i = e % d;        // column-major position of element (i, j)
    double2 v;
    if (k < 5) {
      v = D5[((size_t)x * 5 + k) * bsz + (size_t)i * d + j];
    } else {
      const int mu = k - 5;
      const int nb = nbr9[x * 9 + k];
      v = cconj(D5[((size_t)nb * 5 + 1 + mu) * bsz + (size_t)j * d + i]);
      if ((i < h) != (j < h)) v = mk<double>(-v.x, -v.y);
    }
    o[e] = store_as<S>(v);
  }
}

template <typename S>
void expand_coarse(const double2* D5, const int* nbr9, int V, int d, S* K, hipStream_t s) {
  dim3 grid(V, 9);
  k_expand<S><<<grid, 256, 0, s>>>(D5, nbr9, d, K);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Site kernels: one workgroup of eight wavefronts per site.  Wavefront w
// owns columns w*NCH .. w*NCH+NCH-1 of the nine blocks, lane i the row i;
// the nine input vectors of the site sit in LDS (broadcast reads) and the
// eight partial rows are summed through LDS.  Every load of a block group is
// in flight at once and the code stays compact.  A workgroup serves RB
// right-hand sides of the batch (fields n apart): the block entries it
// loads are applied to all of them.
// ---------------------------------------------------------------------------
constexpr int SW = 8;   // wavefronts per site workgroup

// The block columns of one wavefront: prefetch() issues the loads of the
// first block group (all nine blocks in FP32) into registers, so a kernel can
// start them before it waits for its LDS inputs; apply() multiplies them
// (and any further groups) into RB accumulators.
template <typename T, typename S, int NCH, int RB>
struct SiteCols {
  static constexpr int KG = sizeof(T) == 4 ? 9 : 3;
  S m[KG][NCH];
  const S* Kx;
  size_t bsz;
  unsigned mask;
  int j0, lane, d, row;
  __device__ __forceinline__ void load_group(int k0) {
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const bool blk = (mask >> (k0 + kk)) & 1u;
#pragma unroll
      for (int u = 0; u < NCH; ++u) {
        const int j = j0 + u < d ? j0 + u : 0;
        m[kk][u] = blk ? Kx[(k0 + kk) * bsz + (size_t)j * d + row] : szero<S>();
      }
    }
  }
  // lanes past the last row read row 0 and return zero, so every load of a
  // group is unconditional within the wavefront; the block mask and the
  // column bound are wavefront-uniform
  __device__ __forceinline__ void prefetch(const S* __restrict__ K_, size_t bsz_, unsigned mask_, int j0_, int lane_,
                                           int d_) {
    Kx = K_;
    bsz = bsz_;
    mask = mask_;
    j0 = j0_;
    lane = lane_;
    d = d_;
    row = lane < d ? lane : 0;
    load_group(0);
  }
  __device__ __forceinline__ void apply(const C<T> (*vin)[9][64], C<T> (&acc)[RB]) {
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = czero<T>();
#pragma unroll 1
    for (int k0 = 0; k0 < 9; k0 += KG) {
      if (k0 > 0) load_group(k0);
#pragma unroll
      for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int u = 0; u < NCH; ++u)
          // masked blocks are skipped, not multiplied by zero: their LDS
          // inputs are not loaded and may hold anything
          if (((mask >> (k0 + kk)) & 1u) && j0 + u < d) {
            const C<T> mv = ldc<T, S>(m[kk][u]);
#pragma unroll
            for (int r = 0; r < RB; ++r) cfma(acc[r], mv, vin[r][k0 + kk][j0 + u]);
          }
    }
    // lanes past the last row return zero (callers reduce over all 64 lanes)
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (lane >= d) acc[r] = czero<T>();
  }
};

template <typename T, typename S, int NCH, int RB>
__device__ __forceinline__ void site_cols(const S* __restrict__ Kx, size_t bsz, const C<T> (*vin)[9][64],
                                          unsigned mask, int j0, int lane, int d, C<T> (&acc)[RB]) {
  SiteCols<T, S, NCH, RB> sc;
  sc.prefetch(Kx, bsz, mask, j0, lane, d);
  sc.apply(vin, acc);
}

// sum of the eight wavefronts' partial rows; valid in wavefront 0, lane < d
template <typename T, int RB>
__device__ inline void site_rows_sum(C<T> (&part)[RB], C<T> (*prow)[RB][64]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < RB; ++r) prow[w][r][lane] = part[r];
  __syncthreads();
  if (w == 0)
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      C<T> s = czero<T>();
#pragma unroll
      for (int v = 0; v < SW; ++v) s = cadd(s, prow[v][r][lane]);
      part[r] = s;
    }
}

template <typename T, typename S, int NCH, int RB>
__global__ void __launch_bounds__(64 * SW) k_capply(CoarseOpView<T, S> op, const C<T>* __restrict__ in,
                                                    C<T>* __restrict__ out, long long n) {
  __shared__ C<T> vin[RB][9][64];
  __shared__ C<T> prow[SW][RB][64];
  const int site = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  in += (long long)blockIdx.y * RB * n;
  out += (long long)blockIdx.y * RB * n;
  const size_t bsz = (size_t)d * d;
  SiteCols<T, S, NCH, RB> sc;
  sc.prefetch(op.K + (size_t)site * 9 * bsz, bsz, 0x1FFu, w * NCH, lane, d);
  for (int e = threadIdx.x; e < RB * 9 * d; e += blockDim.x) {
    const int r = e / (9 * d), kj = e % (9 * d);
    vin[r][kj / d][kj % d] = in[r * n + (size_t)op.nbr9[site * 9 + kj / d] * d + kj % d];
  }
  __syncthreads();
  C<T> acc[RB];
  sc.apply(vin, acc);
  site_rows_sum<T, RB>(acc, prow);
  if (w == 0 && lane < d)
#pragma unroll
    for (int r = 0; r < RB; ++r) out[r * n + (size_t)site * d + lane] = acc[r];
}

// ---------------------------------------------------------------------------
// Batched apply on the matrix cores (FP32 arithmetic, 8..16 right-hand
// sides per launch chunk).  Per site the product is a complex GEMM
//   out (d x nb) = [K_0 .. K_8] (d x 9d)  *  [in(nbr_0); ..; in(nbr_8)] (9d x nb),
// done as real 16x16x4 MFMA tiles: rows i of a 16-row tile, RHS r in the
// 16 columns, four complex GEMM columns per step and four real products per
// step (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br).  Wavefront w handles row
// tile w / 3 against block group w % 3 (blocks 3g .. 3g+2); the three
// partial tiles are summed through LDS.  The B operand (the nine input
// vectors of the site for every RHS, [9d][16] complex) is staged in LDS.
// Operand layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; result register v of lane l is D[4 (l / 16) + v][l % 16].
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int MFMA_NB = 16;        // right-hand sides per launch chunk
constexpr int MFMA_MAXD = 56;      // B tile [9d][16] complex within 64 KiB of LDS

template <typename S, int NJ>
__global__ void __launch_bounds__(64 * 12) k_capply_mfma(CoarseOpView<float, S> op, const float2* __restrict__ in,
                                                         float2* __restrict__ out, long long n, int nb) {
  extern __shared__ float2 lds_b[];   // [9d][16] B tile; reused for the partial tiles
  const int site = blockIdx.x, d = op.d;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nmt = (d + 15) >> 4;
  in += (long long)blockIdx.y * MFMA_NB * n;
  out += (long long)blockIdx.y * MFMA_NB * n;
  const int nr = min(MFMA_NB, nb - (int)blockIdx.y * MFMA_NB);
  for (int e = threadIdx.x; e < 9 * d * MFMA_NB; e += blockDim.x) {
    const int j = e / MFMA_NB, r = e % MFMA_NB, k = j / d, jj = j % d;
    lds_b[e] = r < nr ? in[r * n + (size_t)op.nbr9[site * 9 + k] * d + jj] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
  const int mt = w / 3, g = w % 3;
  if (mt < nmt) {
    const int i = mt * 16 + (lane & 15);
    const bool iv = i < d;
    const int ic = iv ? i : 0;
    const int kk = lane >> 4, rl = lane & 15;
    const size_t bsz = (size_t)d * d;
#pragma unroll 1
    for (int k = 3 * g; k < 3 * g + 3; ++k) {
      const S* Kb = op.K + ((size_t)site * 9 + k) * bsz + ic;
      S a[NJ];
#pragma unroll
      for (int t = 0; t < NJ; ++t) a[t] = Kb[(size_t)(4 * t + kk) * d];
      const float2* bt = lds_b + (size_t)(k * d + kk) * MFMA_NB + rl;
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        float2 av = ldc<float, S>(a[t]);
        if (!iv) av = make_float2(0.f, 0.f);
        const float2 bv = bt[(size_t)4 * t * MFMA_NB];
        cr = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-av.y, bv.y, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.y, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.x, ci, 0, 0, 0);
      }
    }
  }
  __syncthreads();   // B tile no longer needed: reuse LDS for the partials
  float2* part = lds_b;   // [3][nmt][16 rows][16 rhs]
  if (mt < nmt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * (lane >> 4) + v;
      part[((size_t)(g * nmt + mt) * 16 + row) * 16 + (lane & 15)] = make_float2(cr[v], ci[v]);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nmt * 16 * 16; e += blockDim.x) {
    const int mtile = e / 256, row = (e / 16) % 16, r = e % 16;
    const int i = mtile * 16 + row;
    if (i < d && r < nr) {
      float2 sum = part[((size_t)(0 * nmt + mtile) * 16 + row) * 16 + r];
      sum = cadd(sum, part[((size_t)(1 * nmt + mtile) * 16 + row) * 16 + r]);
      sum = cadd(sum, part[((size_t)(2 * nmt + mtile) * 16 + row) * 16 + r]);
      out[r * n + (size_t)site * d + i] = sum;
    }
  }
}

template <int LO, int HI, typename F>
inline void with_int(int v, F&& f) {
  if constexpr (LO <= HI) {
    if (v == LO) f(std::integral_constant<int, LO>{});
    else with_int<LO + 1, HI>(v, f);
  } else {
    throw Error(-1, "unsupported size");
  }
}

// whether the matrix-core path takes a batch of nb on d components
inline bool use_mfma(int d, int nb) { return nb >= 8 && d % 4 == 0 && d <= MFMA_MAXD; }

template <typename S>
void coarse_apply_mfma(const CoarseOpView<float, S>& op, const float2* in, float2* out, hipStream_t s, int nb) {
  const long long n = (long long)op.V * op.d;
  const int nmt = (op.d + 15) / 16;
  const size_t lds = std::max((size_t)9 * op.d * MFMA_NB, (size_t)3 * nmt * 256) * sizeof(float2);
  const int nch = (nb + MFMA_NB - 1) / MFMA_NB;
  with_int<1, MFMA_MAXD / 4>(op.d / 4, [&](auto nj) {
    k_capply_mfma<S, decltype(nj)::value><<<dim3(op.V, nch), 64 * 3 * nmt, lds, s>>>(op, in, out, n, nb);
  });
  DD_LAUNCH_CHECK();
}

template <typename T, typename S>
void coarse_apply(const CoarseOpView<T, S>& op, const C<T>* in, C<T>* out, hipStream_t s, int nb) {
  if constexpr (std::is_same<T, float>::value) {
    if (use_mfma(op.d, nb)) {
      coarse_apply_mfma<S>(op, in, out, s, nb);
      return;
    }
  }
  const long long n = (long long)op.V * op.d;
  with_nch(op.d, [&](auto nch) {
    constexpr int NCH = decltype(nch)::value;
    rhs_chunks<T>(nb, [&](auto rb, int first, int nc) {
      constexpr int RB = decltype(rb)::value;
      k_capply<T, S, NCH, RB><<<dim3(op.V, nc), 64 * SW, 0, s>>>(op, in + first * n, out + first * n, n);
    });
  });
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// SAP colour pass as a sequence of site kernels (kernel boundaries are the
// block-wide synchronisation points of MR):
//   k_sap_res:  rho_0 = r = b - D z                       on the sites of colour c
//   k_sap_q(t): alpha_{t-1} from the block inner products of step t-1,
//               rho_t = rho_{t-1} - alpha q_{t-1} (own and in-block neighbour
//               sites, recomputed locally), z += alpha rho_{t-1};
//               q_t = D_i rho_t, per-site <q_t, rho_t>, <q_t, q_t>
//   k_sap_fin:  z += alpha_{last} rho_{last}
// Buffers rho, q, part are ping-ponged by step parity.  Vectors of the batch
// are n apart, per-site partials V*4 apart.  The per-site partials are
// stored block-major (position pos(x) = block * bs + index in block) so that
// a block's step size is one contiguous read, and each site's in-block
// neighbour mask is a table: no kernel chases an index to find another.
// The operator blocks are loaded before the kernel waits for its inputs.
// ---------------------------------------------------------------------------
template <typename T, typename S, int NCH, int RB>
__global__ void __launch_bounds__(64 * SW) k_sap_res(CoarseOpView<T, S> op, const int* __restrict__ csites,
                                                     const C<T>* __restrict__ b, const C<T>* __restrict__ z,
                                                     C<T>* __restrict__ rho0, long long n) {
  __shared__ C<T> vin[RB][9][64];
  __shared__ C<T> prow[SW][RB][64];
  const int site = csites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  const long long off = (long long)blockIdx.y * RB * n;
  b += off;
  z += off;
  rho0 += off;
  const size_t bsz = (size_t)d * d;
  SiteCols<T, S, NCH, RB> sc;
  sc.prefetch(op.K + (size_t)site * 9 * bsz, bsz, 0x1FFu, w * NCH, lane, d);
  for (int e = threadIdx.x; e < RB * 9 * d; e += blockDim.x) {
    const int r = e / (9 * d), kj = e % (9 * d);
    vin[r][kj / d][kj % d] = z[r * n + (size_t)op.nbr9[site * 9 + kj / d] * d + kj % d];
  }
  __syncthreads();
  C<T> acc[RB];
  sc.apply(vin, acc);
  site_rows_sum<T, RB>(acc, prow);
  if (w == 0 && lane < d)
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const size_t o = r * n + (size_t)site * d + lane;
      rho0[o] = csub(b[o], acc[r]);
    }
}

// block step size from the block-major per-site partials of one block,
// summed by one wavefront (lane v takes sites v, v+64, ..) in a fixed order;
// every lane of the wavefront gets the result
template <typename T>
__device__ inline C<T> block_alpha_wave(const T* __restrict__ part, int blk, int bs, int lane) {
  T s0 = 0, s1 = 0, s2 = 0;
  for (int v = lane; v < bs; v += 64) {
    const T* p = part + ((size_t)blk * bs + v) * 4;
    s0 += p[0];
    s1 += p[1];
    s2 += p[2];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  return s2 > T(0) ? mk<T>(s0 / s2, s1 / s2) : czero<T>();
}

// The workgroup of the site at position pos0 + blockIdx.x of the block-major
// order (blk_sites and site_pos are inverse tables) finds its block and its
// in-block mask without chasing the site index; the inputs of the step are
// read before the step size of the previous step is known, which is then
// applied to them in registers.
template <typename T, typename S, int NCH, int RB>
__global__ void __launch_bounds__(64 * SW) k_sap_q(CoarseOpView<T, S> op, const int* __restrict__ csites,
                                                   SapTables tb, int pos0, int step,
                                                   const C<T>* __restrict__ rho_prev, const C<T>* __restrict__ q_prev,
                                                   const T* __restrict__ part_prev, C<T>* __restrict__ rho_cur,
                                                   C<T>* __restrict__ q_cur, T* __restrict__ part_cur,
                                                   C<T>* __restrict__ z, long long n) {
  __shared__ C<T> vin[RB][9][64];
  __shared__ C<T> prow[SW][RB][64];
  __shared__ C<T> alpha_s[RB];
  const int site = csites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  const long long off = (long long)blockIdx.y * RB * n, pn = (long long)op.V * 4;
  const long long poff = (long long)blockIdx.y * RB * pn;
  rho_prev += off;
  q_prev += off;
  rho_cur += off;
  q_cur += off;
  z += off;
  part_prev += poff;
  part_cur += poff;
  const int pos = pos0 + blockIdx.x, blk = pos / tb.bs;
  if (step > 0 && w < RB) {
    const C<T> a = block_alpha_wave<T>(part_prev + w * pn, blk, tb.bs, lane);
    if (lane == 0) alpha_s[w] = a;
  }
  const unsigned mask = tb.inmask[pos];   // self and the in-block neighbours
  const size_t bsz = (size_t)d * d;
  SiteCols<T, S, NCH, RB> sc;
  sc.prefetch(op.K + (size_t)site * 9 * bsz, bsz, mask, w * NCH, lane, d);
  // this thread's share of the in-block inputs, and the site's own z and
  // previous residual for the update of z
  constexpr int EPT = (RB * 9 * 64 + 64 * SW - 1) / (64 * SW);
  C<T> rv[EPT], qv[EPT];
  int slot[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * 64 * SW;
    slot[i] = -1;
    rv[i] = qv[i] = czero<T>();
    if (e < RB * 9 * d) {
      const int r = e / (9 * d), k = (e % (9 * d)) / d, j = e % d;
      if ((mask >> k) & 1u) {
        const size_t o = r * n + (size_t)op.nbr9[site * 9 + k] * d + j;
        rv[i] = rho_prev[o];
        if (step > 0) qv[i] = q_prev[o];
        slot[i] = e;
      }
    }
  }
  C<T> zown[RB], rown[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    zown[r] = rown[r] = czero<T>();
    if (step > 0 && w == 0 && lane < d) {
      const size_t o = r * n + (size_t)site * d + lane;
      zown[r] = z[o];
      rown[r] = rho_prev[o];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (slot[i] >= 0) {
      const int e = slot[i], r = e / (9 * d), k = (e % (9 * d)) / d, j = e % d;
      C<T> v = rv[i];
      if (step > 0) v = csub(v, cmul(alpha_s[r], qv[i]));
      vin[r][k][j] = v;
    }
  __syncthreads();
  C<T> q[RB];
  sc.apply(vin, q);
  site_rows_sum<T, RB>(q, prow);
  if (w == 0) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      C<T> rho = czero<T>();
      if (lane < d) {
        const size_t o = r * n + (size_t)site * d + lane;
        rho = vin[r][0][lane];
        rho_cur[o] = rho;
        q_cur[o] = q[r];
        if (step > 0) {
          cfma(zown[r], alpha_s[r], rown[r]);
          z[o] = zown[r];
        }
      }
      const C<T> qq = lane < d ? q[r] : czero<T>();
      T a0 = qq.x * rho.x + qq.y * rho.y, a1 = qq.x * rho.y - qq.y * rho.x, a2 = qq.x * qq.x + qq.y * qq.y;
      a0 = wave_sum(a0);
      a1 = wave_sum(a1);
      a2 = wave_sum(a2);
      if (lane == 0) {
        T* p = part_cur + r * pn + (size_t)pos * 4;
        p[0] = a0;
        p[1] = a1;
        p[2] = a2;
      }
    }
  }
}

// The MR step of one field in FP32 arithmetic for blocks in which no site
// has more than KM of its nine operator blocks inside (2^4 blocks: itself and
// four neighbours).  Four wavefronts per site, wavefront w owning columns
// w*NCH .. w*NCH+NCH-1, lane i the row i; the prefetch registers hold only
// the blocks the site reads (the mask's set bits in order), so that per
// register twice the operator bytes of k_sap_q's nine-block layout are in
// flight: the step is bound by the loads a compute unit keeps outstanding.
constexpr int SW4 = 4;
template <typename S, int NCH, int KM>
__global__ void __launch_bounds__(64 * SW4) k_sap_q1(CoarseOpView<float, S> op, const int* __restrict__ csites,
                                                     SapTables tb, int pos0, int step,
                                                     const float2* __restrict__ rho_prev,
                                                     const float2* __restrict__ q_prev,
                                                     const float* __restrict__ part_prev, float2* __restrict__ rho_cur,
                                                     float2* __restrict__ q_cur, float* __restrict__ part_cur,
                                                     float2* __restrict__ z, long long n) {
  __shared__ float2 vin[9][64];
  __shared__ float2 prow[SW4][64];
  __shared__ float2 alpha_s;
  const int site = csites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  const long long off = (long long)blockIdx.y * n, poff = (long long)blockIdx.y * op.V * 4;
  rho_prev += off;
  q_prev += off;
  rho_cur += off;
  q_cur += off;
  z += off;
  part_prev += poff;
  part_cur += poff;
  const int pos = pos0 + blockIdx.x, blk = pos / tb.bs;
  if (step > 0 && w == 0) {
    const float2 a = block_alpha_wave<float>(part_prev, blk, tb.bs, lane);
    if (lane == 0) alpha_s = a;
  }
  const unsigned mask = tb.inmask[pos];
  int kb[KM];
  {
    unsigned mm = mask;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
      kb[kk] = mm ? __builtin_ctz(mm) : -1;
      mm &= mm - 1u;
    }
  }
  const size_t bsz = (size_t)d * d;
  const S* Kx = op.K + (size_t)site * 9 * bsz;
  const int j0 = w * NCH, row = lane < d ? lane : 0;
  S m[KM][NCH];
#pragma unroll
  for (int kk = 0; kk < KM; ++kk)
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      const int j = j0 + u < d ? j0 + u : 0;
      m[kk][u] = kb[kk] >= 0 ? Kx[kb[kk] * bsz + (size_t)j * d + row] : szero<S>();
    }
  constexpr int EPT = (9 * 64 + 64 * SW4 - 1) / (64 * SW4);
  float2 rv[EPT], qv[EPT];
  int slot[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * 64 * SW4;
    slot[i] = -1;
    rv[i] = qv[i] = czero<float>();
    if (e < 9 * d) {
      const int k = e / d, j = e % d;
      if ((mask >> k) & 1u) {
        const size_t o = (size_t)op.nbr9[site * 9 + k] * d + j;
        rv[i] = rho_prev[o];
        if (step > 0) qv[i] = q_prev[o];
        slot[i] = e;
      }
    }
  }
  float2 zown = czero<float>(), rown = czero<float>();
  const size_t own = (size_t)site * d + lane;
  if (step > 0 && w == 0 && lane < d) {
    zown = z[own];
    rown = rho_prev[own];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (slot[i] >= 0) {
      const int e = slot[i];
      float2 v = rv[i];
      if (step > 0) v = csub(v, cmul(alpha_s, qv[i]));
      vin[e / d][e % d] = v;
    }
  __syncthreads();
  float2 acc = czero<float>();
#pragma unroll
  for (int kk = 0; kk < KM; ++kk)
    if (kb[kk] >= 0)
#pragma unroll
      for (int u = 0; u < NCH; ++u)
        if (j0 + u < d) cfma(acc, ldc<float, S>(m[kk][u]), vin[kb[kk]][j0 + u]);
  if (lane >= d) acc = czero<float>();
  prow[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    float2 q = czero<float>(), rho = czero<float>();
#pragma unroll
    for (int v = 0; v < SW4; ++v) q = cadd(q, prow[v][lane]);
    if (lane < d) {
      rho = vin[0][lane];
      rho_cur[own] = rho;
      q_cur[own] = q;
      if (step > 0) {
        cfma(zown, alpha_s, rown);
        z[own] = zown;
      }
    } else {
      q = czero<float>();
    }
    float a0 = q.x * rho.x + q.y * rho.y, a1 = q.x * rho.y - q.y * rho.x, a2 = q.x * q.x + q.y * q.y;
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      float* p = part_cur + (size_t)pos * 4;
      p[0] = a0;
      p[1] = a1;
      p[2] = a2;
    }
  }
}

// columns per wavefront of k_sap_q1 for d components: an even number
template <typename F>
inline void with_nch4(int d, F&& f) {
  switch ((d + 7) / 8) {
    case 1: f(std::integral_constant<int, 2>{}); break;
    case 2: f(std::integral_constant<int, 4>{}); break;
    case 3: f(std::integral_constant<int, 6>{}); break;
    case 4: f(std::integral_constant<int, 8>{}); break;
    case 5: f(std::integral_constant<int, 10>{}); break;
    case 6: f(std::integral_constant<int, 12>{}); break;
    case 7: f(std::integral_constant<int, 14>{}); break;
    case 8: f(std::integral_constant<int, 16>{}); break;
    default: throw Error(-1, "coarse levels support at most 64 components per site");
  }
}
// k_sap_q1 takes the step when the arithmetic is FP32, the field is one,
// every site reads at most five blocks and their prefetch fits 80 registers
constexpr int Q1_KM = 5;
template <typename T, typename S>
inline bool use_sap_q1(const SapTables& tb, int d) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    const int nch4 = 2 * ((d + 7) / 8);
    return tb.kmax <= Q1_KM && Q1_KM * nch4 * (int)(sizeof(S) / 4) <= 80;
  }
}

template <typename T>
__global__ void k_sap_fin(int d, const int* __restrict__ csites, SapTables tb, int pos0,
                          const C<T>* __restrict__ rho, const T* __restrict__ part, C<T>* __restrict__ z, long long n,
                          long long pn) {
  __shared__ C<T> alpha_s;
  const int site = csites[blockIdx.x];
  const int blk = (pos0 + blockIdx.x) / tb.bs;
  rho += blockIdx.y * n;
  z += blockIdx.y * n;
  part += blockIdx.y * pn;
  if (threadIdx.x < 64) {
    const C<T> a = block_alpha_wave<T>(part, blk, tb.bs, threadIdx.x);
    if (threadIdx.x == 0) alpha_s = a;
  }
  const int i = threadIdx.x;
  C<T> zz = czero<T>(), rr = czero<T>();
  const size_t o = (size_t)site * d + i;
  if (i < d) {
    zz = z[o];
    rr = rho[o];
  }
  __syncthreads();
  if (i < d) {
    cfma(zz, alpha_s, rr);
    z[o] = zz;
  }
}

template <typename T, typename S>
void coarse_sap_colour(const CoarseOpView<T, S>& op, const SapTables& tb, int colour, int mr_iters, const C<T>* b,
                       C<T>* z, SapScratch<T>& ws, hipStream_t s, int nb) {
  if (mr_iters <= 0) return;
  DD_REQUIRE(op.d <= 64, "coarse levels support at most 64 components per site");
  const int nsites = (tb.nblk / 2) * tb.bs;
  const int pos0 = colour * (tb.nblk / 2) * tb.bs;   // blocks are colour-major
  const int* csites = tb.blk_sites + pos0;
  const long long n = (long long)op.V * op.d, pn = (long long)op.V * 4;
  with_nch(op.d, [&](auto nch) {
    constexpr int NCH = decltype(nch)::value;
    rhs_chunks<T>(nb, [&](auto rb, int first, int nc) {
      constexpr int RB = decltype(rb)::value;
      const long long o = first * n, po = first * pn;
      // the residual is rho_0 and lands in the "previous" buffer of step 0
      k_sap_res<T, S, NCH, RB><<<dim3(nsites, nc), 64 * SW, 0, s>>>(op, csites, b + o, z + o, ws.rho[1] + o, n);
      for (int t = 0; t < mr_iters; ++t) {
        const int pp = (t + 1) & 1, cc = t & 1;   // previous / current buffers
        if constexpr (RB == 1 && std::is_same<T, float>::value) {
          if (use_sap_q1<T, S>(tb, op.d)) {
            with_nch4(op.d, [&](auto nch4) {
              constexpr int NC4 = decltype(nch4)::value;
              if constexpr (Q1_KM * NC4 * (int)(sizeof(S) / 4) <= 80) {
                k_sap_q1<S, NC4, Q1_KM><<<dim3(nsites, nc), 64 * SW4, 0, s>>>(
                    op, csites, tb, pos0, t, ws.rho[pp] + o, ws.q[pp] + o, ws.part[pp] + po, ws.rho[cc] + o,
                    ws.q[cc] + o, ws.part[cc] + po, z + o, n);
              }
            });
            continue;
          }
        }
        k_sap_q<T, S, NCH, RB><<<dim3(nsites, nc), 64 * SW, 0, s>>>(
            op, csites, tb, pos0, t, ws.rho[pp] + o, ws.q[pp] + o, ws.part[pp] + po, ws.rho[cc] + o, ws.q[cc] + o,
            ws.part[cc] + po, z + o, n);
      }
    });
  });
  const int last = (mr_iters - 1) & 1;
  k_sap_fin<T><<<dim3(nsites, nb), 64 * ((op.d + 63) / 64), 0, s>>>(op.d, csites, tb, pos0, ws.rho[last],
                                                                   ws.part[last], z, n, pn);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// odd-even building blocks (site workgroups, as above)
// ---------------------------------------------------------------------------
template <typename T, typename S, int NCH, int RB>
__global__ void __launch_bounds__(64 * SW) k_csites(CoarseOpView<T, S> op, const int* __restrict__ sites,
                                                    T gamma, const C<T>* __restrict__ in_c, T alpha,
                                                    const C<T>* __restrict__ in_s, T beta,
                                                    const C<T>* __restrict__ in_h, C<T>* __restrict__ out,
                                                    long long n) {
  __shared__ C<T> vin[RB][9][64];
  __shared__ C<T> prow[SW][RB][64];
  const int site = sites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  const long long off = (long long)blockIdx.y * RB * n;
  unsigned mask = 0;
  if (alpha != T(0)) mask |= 1u;
  if (beta != T(0)) mask |= 0x1FEu;
  const size_t bsz = (size_t)d * d;
  SiteCols<T, S, NCH, RB> sc;
  sc.prefetch(op.K + (size_t)site * 9 * bsz, bsz, mask, w * NCH, lane, d);
  for (int e = threadIdx.x; e < RB * 9 * d; e += blockDim.x) {
    const int r = e / (9 * d), kj = e % (9 * d), k = kj / d, j = kj % d;
    if ((mask >> k) & 1u) {
      const C<T> v = (k == 0 ? in_s : in_h)[off + r * n + (size_t)op.nbr9[site * 9 + k] * d + j];
      vin[r][k][j] = k == 0 ? cscale(v, alpha) : cscale(v, beta);
    }
  }
  __syncthreads();
  C<T> acc[RB];
  sc.apply(vin, acc);
  site_rows_sum<T, RB>(acc, prow);
  if (w == 0 && lane < d)
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const size_t o = off + r * n + (size_t)site * d + lane;
      C<T> a = acc[r];
      if (gamma != T(0)) a = cadd(a, cscale(in_c[o], gamma));
      out[o] = a;
    }
}

template <typename T, typename S>
void coarse_site_apply(const CoarseOpView<T, S>& op, const int* sites, int nsites, T gamma,
                       const C<T>* in_c, T alpha, const C<T>* in_s, T beta, const C<T>* in_h,
                       C<T>* out, hipStream_t s, int nb) {
  const long long n = (long long)op.V * op.d;
  with_nch(op.d, [&](auto nch) {
    constexpr int NCH = decltype(nch)::value;
    rhs_chunks<T>(nb, [&](auto rb, int first, int nc) {
      constexpr int RB = decltype(rb)::value;
      const long long o = first * n;
      k_csites<T, S, NCH, RB><<<dim3(nsites, nc), 64 * SW, 0, s>>>(
          op, sites, gamma, in_c ? in_c + o : nullptr, alpha, in_s ? in_s + o : nullptr, beta,
          in_h ? in_h + o : nullptr, out + o, n);
    });
  });
  DD_LAUNCH_CHECK();
}

template <typename T, int NCH, int RB>
__global__ void __launch_bounds__(64 * SW) k_site_matvec(const C<T>* __restrict__ M,
                                                         const int* __restrict__ sites, int d,
                                                         const C<T>* __restrict__ in, C<T>* __restrict__ out,
                                                         long long n) {
  __shared__ C<T> vin[RB][9][64];
  __shared__ C<T> prow[SW][RB][64];
  const int k = blockIdx.x, site = sites[k], w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long off = (long long)blockIdx.y * RB * n;
  for (int e = threadIdx.x; e < RB * d; e += blockDim.x)
    vin[e / d][0][e % d] = in[off + (e / d) * n + (size_t)site * d + e % d];
  __syncthreads();
  C<T> acc[RB];
  site_cols<T, C<T>, NCH, RB>(M + (size_t)k * d * d, (size_t)d * d, vin, 1u, w * NCH, lane, d, acc);
  site_rows_sum<T, RB>(acc, prow);
  if (w == 0 && lane < d)
#pragma unroll
    for (int r = 0; r < RB; ++r) out[off + r * n + (size_t)site * d + lane] = acc[r];
}

template <typename T>
void site_matvec(const C<T>* M, const int* sites, int nsites, int d, long long n, const C<T>* in, C<T>* out,
                 hipStream_t s, int nb) {
  with_nch(d, [&](auto nch) {
    constexpr int NCH = decltype(nch)::value;
    rhs_chunks<T>(nb, [&](auto rb, int first, int nc) {
      constexpr int RB = decltype(rb)::value;
      k_site_matvec<T, NCH, RB><<<dim3(nsites, nc), 64 * SW, 0, s>>>(M, sites, d, in + first * n,
                                                                     out + first * n, n);
    });
  });
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// dense Schur complement of a small coarsest level: the workgroup first
// stages the odd components of its RB input fields in LDS (one gather through
// the index table), then each wavefront takes one row, its lanes striding
// over the row (contiguous) against the staged input; four rows per
// workgroup
// ---------------------------------------------------------------------------
template <typename T, int RB>
__global__ void __launch_bounds__(256) k_dense_schur(const C<T>* __restrict__ S, int m,
                                                     const int* __restrict__ oidx, const int* __restrict__ eidx,
                                                     const C<T>* __restrict__ in, C<T>* __restrict__ out,
                                                     long long n) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* vs = reinterpret_cast<C<T>*>(smem_raw);   // [RB][m]
  const long long off = (long long)blockIdx.y * RB * n;
  in += off;
  out += off;
  for (int e = threadIdx.x; e < RB * m; e += blockDim.x) {
    const int r = e / m, j = e - r * m;
    vs[e] = in[r * n + oidx[j]];
  }
  __syncthreads();
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= m) return;   // after the only barrier; wavefront-uniform
  const C<T>* row = S + (size_t)i * m;
  C<T> acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = czero<T>();
#pragma unroll 4
  for (int j = lane; j < m; j += 64) {
    const C<T> a = row[j];
#pragma unroll
    for (int r = 0; r < RB; ++r) cfma(acc[r], a, vs[r * m + j]);
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const T re = wave_sum(acc[r].x), im = wave_sum(acc[r].y);
    if (lane == 0) {
      out[r * n + oidx[i]] = mk<T>(re, im);
      out[r * n + eidx[i]] = czero<T>();
    }
  }
}

// the staged input is RB * m elements: at most 64 KiB for m <= 2048 (FP32
// with four fields, FP64 with two), within the default dynamic LDS limit
template <typename T>
void dense_schur_apply(const C<T>* S, int m, const int* oidx, const int* eidx, long long n, const C<T>* in,
                       C<T>* out, hipStream_t s, int nb) {
  DD_REQUIRE(m >= 1 && (long long)m <= n && m <= 2048, "bad dense Schur shape");
  rhs_chunks<T>(nb, [&](auto rb, int first, int nc) {
    constexpr int RB = decltype(rb)::value;
    const size_t sm = (size_t)RB * m * sizeof(C<T>);
    k_dense_schur<T, RB><<<dim3((m + 3) / 4, nc), 256, sm, s>>>(S, m, oidx, eidx, in + first * n,
                                                               out + first * n, n);
  });
  DD_LAUNCH_CHECK();
}

__global__ void k_schur_unit_cols(double2* __restrict__ e, long long n, int nbc, const int* __restrict__ oidx,
                                  int j0) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nbc) return;
  const int r = (int)(t / n);
  const long long k = t - (long long)r * n;
  e[t] = make_double2(k == oidx[j0 + r] ? 1.0 : 0.0, 0.0);
}

void schur_unit_cols(double2* e, long long n, int nbc, const int* oidx, int j0, hipStream_t s) {
  const long long tot = n * nbc;
  k_schur_unit_cols<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(e, n, nbc, oidx, j0);
  DD_LAUNCH_CHECK();
}

__global__ void k_schur_gather_cols(const double2* __restrict__ cols, long long n, int nbc,
                                    const int* __restrict__ oidx, int m, int j0, double2* __restrict__ S) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * nbc) return;
  const int i = (int)(t / nbc), r = (int)(t % nbc);
  S[(size_t)i * m + j0 + r] = cols[r * n + oidx[i]];
}

void schur_gather_cols(const double2* cols, long long n, int nbc, const int* oidx, int m, int j0, double2* S,
                       hipStream_t s) {
  const long long tot = (long long)m * nbc;
  k_schur_gather_cols<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(cols, n, nbc, oidx, m, j0, S);
  DD_LAUNCH_CHECK();
}

// Gauss-Jordan inversion of the self block of every listed site, FP64.
__global__ void k_self_inverse(const double2* __restrict__ D5, const int* __restrict__ sites, int d,
                               double2* __restrict__ inv, int* __restrict__ flag) {
  extern __shared__ unsigned char smem_raw[];
  double2* a = reinterpret_cast<double2*>(smem_raw);     // [d][2d]
  __shared__ int piv;
  __shared__ double2 fcol[64];   // the pivot column's multipliers of one step
  const int k = blockIdx.x, site = sites[k];
  const int w = 2 * d;
  const double2* S = D5 + (size_t)site * 5 * d * d;
  for (int e = threadIdx.x; e < d * w; e += blockDim.x) {
    const int r = e / w, c = e % w;
    a[e] = c < d ? S[(size_t)r * d + c] : mk<double>(c - d == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int col = 0; col < d; ++col) {
    if (threadIdx.x == 0) {
      int best = col;
      double bv = -1.0;
      for (int r = col; r < d; ++r) {
        const double2 v = a[r * w + col];
        const double m = v.x * v.x + v.y * v.y;
        if (m > bv) { bv = m; best = r; }
      }
      piv = best;
    }
    __syncthreads();
    if (piv != col)
      for (int c = threadIdx.x; c < w; c += blockDim.x) {
        double2 tmp = a[col * w + c];
        a[col * w + c] = a[piv * w + c];
        a[piv * w + c] = tmp;
      }
    __syncthreads();
    const double2 p = a[col * w + col];
    const double pn = p.x * p.x + p.y * p.y;
    if (threadIdx.x == 0 && !(pn > 0.0 && pn < INFINITY)) *flag = 1;   // singular or non-finite block
    const double2 pinv = mk<double>(p.x / pn, -p.y / pn);
    __syncthreads();
    for (int c = threadIdx.x; c < w; c += blockDim.x) a[col * w + c] = cmul(a[col * w + c], pinv);
    // every row's multiplier is read before any row is updated: the update
    // of row r overwrites a[r][col], which the other elements of the row
    // still need (a row spans several wavefronts and loop trips)
    for (int r = threadIdx.x; r < d; r += blockDim.x) fcol[r] = a[r * w + col];
    __syncthreads();
    for (int e = threadIdx.x; e < d * w; e += blockDim.x) {
      const int r = e / w, c = e % w;
      if (r != col) a[e] = csub(a[e], cmul(fcol[r], a[col * w + c]));
    }
    __syncthreads();
  }
  // column-major result: element (r, c) at c*d + r
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int c = e / d, r = e % d;
    inv[(size_t)k * d * d + e] = a[r * w + d + c];
  }
}

void self_block_inverse(const double2* D, const int* sites, int nsites, int d, double2* inv, int* flag,
                        hipStream_t s) {
  DD_REQUIRE(d >= 1 && d <= 64, "self-block inversion supports at most 64 components per site");
  const size_t sm = (size_t)d * 2 * d * sizeof(double2);
  DD_CHECK_HIP(hipFuncSetAttribute((const void*)k_self_inverse,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm));
  k_self_inverse<<<nsites, 256, sm, s>>>(D, sites, d, inv, flag);
  DD_LAUNCH_CHECK();
}

// canonical export: [V][9][d][d] row-major
__global__ void k_export_coarse(CoarseOpView<double> op, double2* __restrict__ out) {
  const int site = blockIdx.x, k = blockIdx.y;
  const int d = op.d;
  const size_t bsz = (size_t)d * d;
  const double2* src = op.K + ((size_t)site * 9 + k) * bsz;
  double2* o = out + ((size_t)site * 9 + k) * bsz;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int i = e / d, j = e % d;
    o[e] = src[(size_t)j * d + i];
  }
}

void export_coarse(const CoarseOpView<double>& op, double2* out, hipStream_t s) {
  dim3 grid(op.V, 9);
  k_export_coarse<<<grid, 256, 0, s>>>(op, out);
  DD_LAUNCH_CHECK();
}

template void expand_coarse<double2>(const double2*, const int*, int, int, double2*, hipStream_t);
template void expand_coarse<float2>(const double2*, const int*, int, int, float2*, hipStream_t);
template void expand_coarse<__half2>(const double2*, const int*, int, int, __half2*, hipStream_t);

#define DD_INST(T, S)                                                                              \
  template void coarse_apply<T, S>(const CoarseOpView<T, S>&, const C<T>*, C<T>*, hipStream_t, int); \
  template void coarse_sap_colour<T, S>(const CoarseOpView<T, S>&, const SapTables&, int, int, const C<T>*, \
                                        C<T>*, SapScratch<T>&, hipStream_t, int);                    \
  template void coarse_site_apply<T, S>(const CoarseOpView<T, S>&, const int*, int, T, const C<T>*, T, \
                                        const C<T>*, T, const C<T>*, C<T>*, hipStream_t, int);
DD_INST(double, double2)
DD_INST(float, float2)
DD_INST(float, __half2)
#undef DD_INST
template void dense_schur_apply<double>(const double2*, int, const int*, const int*, long long, const double2*,
                                        double2*, hipStream_t, int);
template void dense_schur_apply<float>(const float2*, int, const int*, const int*, long long, const float2*,
                                       float2*, hipStream_t, int);
template void site_matvec<double>(const double2*, const int*, int, int, long long, const double2*, double2*,
                                  hipStream_t, int);
template void site_matvec<float>(const float2*, const int*, int, int, long long, const float2*, float2*,
                                 hipStream_t, int);

}  // namespace ddamg
