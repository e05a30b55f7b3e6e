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
        }
        ++nbk;
      }
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
// in flight at once and the code stays compact.
// ---------------------------------------------------------------------------
constexpr int SW = 8;   // wavefronts per site workgroup

template <typename T, typename S, int NCH>
__device__ __forceinline__ C<T> site_cols(const S* __restrict__ Kx, size_t bsz, const C<T> (*vin)[64],
                                          unsigned mask, int j0, int lane, int d) {
  constexpr int KG = sizeof(T) == 4 ? 9 : 3;
  // lanes past the last row read row 0 and return zero, so every
  // load of a group is unconditional within the wavefront; the block mask
  // and the column bound are wavefront-uniform
  const int row = lane < d ? lane : 0;
  C<T> acc = czero<T>();
#pragma unroll 1
  for (int k0 = 0; k0 < 9; k0 += KG) {
    // raw stored values: all loads issue before the first conversion
    S m[KG][NCH];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const bool blk = (mask >> (k0 + kk)) & 1u;
#pragma unroll
      for (int u = 0; u < NCH; ++u) {
        const int j = j0 + u < d ? j0 + u : 0;
        m[kk][u] = blk ? Kx[(k0 + kk) * bsz + (size_t)j * d + row] : szero<S>();
      }
    }
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
      for (int u = 0; u < NCH; ++u)
        // masked blocks are skipped, not multiplied by zero: their LDS
        // inputs are not loaded and may hold anything
        if (((mask >> (k0 + kk)) & 1u) && j0 + u < d) cfma(acc, ldc<T, S>(m[kk][u]), vin[k0 + kk][j0 + u]);
  }
  // lanes past the last row return zero (callers reduce over all 64 lanes)
  return lane < d ? acc : czero<T>();
}

// sum of the eight wavefronts' partial rows; valid in wavefront 0, lane < d
template <typename T>
__device__ inline C<T> site_rows_sum(C<T> part, C<T> (*prow)[64]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  prow[w][lane] = part;
  __syncthreads();
  C<T> s = czero<T>();
  if (w == 0)
#pragma unroll
    for (int v = 0; v < SW; ++v) s = cadd(s, prow[v][lane]);
  return s;
}

template <typename T, typename S, int NCH>
__global__ void __launch_bounds__(64 * SW) k_capply(CoarseOpView<T, S> op, const C<T>* __restrict__ in,
                                                    C<T>* __restrict__ out) {
  __shared__ C<T> vin[9][64];
  __shared__ C<T> prow[SW][64];
  const int site = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  for (int e = threadIdx.x; e < 9 * d; e += blockDim.x)
    vin[e / d][e % d] = in[(size_t)op.nbr9[site * 9 + e / d] * d + e % d];
  __syncthreads();
  const size_t bsz = (size_t)d * d;
  const C<T> r = site_rows_sum<T>(site_cols<T, S, NCH>(op.K + (size_t)site * 9 * bsz, bsz, vin, 0x1FFu,
                                                     w * NCH, lane, d), prow);
  if (w == 0 && lane < d) out[(size_t)site * d + lane] = r;
}

template <typename T, typename S>
void coarse_apply(const CoarseOpView<T, S>& op, const C<T>* in, C<T>* out, hipStream_t s) {
  with_nch(op.d, [&](auto nch) {
    k_capply<T, S, decltype(nch)::value><<<op.V, 64 * SW, 0, s>>>(op, in, out);
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
// Buffers rho, q, part are ping-ponged by step parity.
// ---------------------------------------------------------------------------
template <typename T, typename S, int NCH>
__global__ void __launch_bounds__(64 * SW) k_sap_res(CoarseOpView<T, S> op, const int* __restrict__ csites,
                                                     const C<T>* __restrict__ b, const C<T>* __restrict__ z,
                                                     C<T>* __restrict__ rho0) {
  __shared__ C<T> vin[9][64];
  __shared__ C<T> prow[SW][64];
  const int site = csites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  for (int e = threadIdx.x; e < 9 * d; e += blockDim.x)
    vin[e / d][e % d] = z[(size_t)op.nbr9[site * 9 + e / d] * d + e % d];
  __syncthreads();
  const size_t bsz = (size_t)d * d;
  const C<T> dz = site_rows_sum<T>(site_cols<T, S, NCH>(op.K + (size_t)site * 9 * bsz, bsz, vin, 0x1FFu,
                                                      w * NCH, lane, d), prow);
  if (w == 0 && lane < d) rho0[(size_t)site * d + lane] = csub(b[(size_t)site * d + lane], dz);
}

// block alpha of step t from the per-site partials of the block's sites
template <typename T>
__device__ inline C<T> block_alpha(const T* __restrict__ part, const int* __restrict__ bsites, int bs) {
  T s0 = 0, s1 = 0, s2 = 0;
  for (int v = 0; v < bs; ++v) {
    const T* p = part + (size_t)bsites[v] * 4;
    s0 += p[0];
    s1 += p[1];
    s2 += p[2];
  }
  return s2 > T(0) ? mk<T>(s0 / s2, s1 / s2) : czero<T>();
}

template <typename T, typename S, int NCH>
__global__ void __launch_bounds__(64 * SW) k_sap_q(CoarseOpView<T, S> op, const int* __restrict__ csites,
                                                   const int* __restrict__ blk_sites,
                                                   const int* __restrict__ site_blk, int bs, int step,
                                                   const C<T>* __restrict__ rho_prev,
                                                   const C<T>* __restrict__ q_prev,
                                                   const T* __restrict__ part_prev, C<T>* __restrict__ rho_cur,
                                                   C<T>* __restrict__ q_cur, T* __restrict__ part_cur,
                                                   C<T>* __restrict__ z) {
  __shared__ C<T> vin[9][64];
  __shared__ C<T> prow[SW][64];
  __shared__ C<T> alpha_s;
  const int site = csites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  const int blk = site_blk[site];
  unsigned mask = 1u;   // self and the in-block neighbours
  for (int k = 1; k < 9; ++k)
    if (site_blk[op.nbr9[site * 9 + k]] == blk) mask |= 1u << k;
  if (step > 0 && threadIdx.x == 0) alpha_s = block_alpha<T>(part_prev, blk_sites + (size_t)blk * bs, bs);
  __syncthreads();
  const C<T> alpha = step > 0 ? alpha_s : czero<T>();
  for (int e = threadIdx.x; e < 9 * d; e += blockDim.x) {
    const int k = e / d, j = e % d;
    if ((mask >> k) & 1u) {
      const size_t o = (size_t)op.nbr9[site * 9 + k] * d + j;
      C<T> r = rho_prev[o];
      if (step > 0) r = csub(r, cmul(alpha, q_prev[o]));
      vin[k][j] = r;
    }
  }
  __syncthreads();
  const size_t bsz = (size_t)d * d;
  const C<T> q = site_rows_sum<T>(site_cols<T, S, NCH>(op.K + (size_t)site * 9 * bsz, bsz, vin, mask,
                                                     w * NCH, lane, d), prow);
  if (w == 0) {
    C<T> rho = czero<T>();
    if (lane < d) {
      const size_t o = (size_t)site * d + lane;
      rho = vin[0][lane];
      rho_cur[o] = rho;
      q_cur[o] = q;
      if (step > 0) {
        C<T> zz = z[o];
        cfma(zz, alpha, rho_prev[o]);
        z[o] = zz;
      }
    }
    T a0 = q.x * rho.x + q.y * rho.y, a1 = q.x * rho.y - q.y * rho.x, a2 = q.x * q.x + q.y * q.y;
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      T* p = part_cur + (size_t)site * 4;
      p[0] = a0;
      p[1] = a1;
      p[2] = a2;
    }
  }
}

template <typename T>
__global__ void k_sap_fin(int d, const int* __restrict__ csites, const int* __restrict__ blk_sites,
                          const int* __restrict__ site_blk, int bs, const C<T>* __restrict__ rho,
                          const T* __restrict__ part, C<T>* __restrict__ z) {
  __shared__ C<T> alpha_s;
  const int site = csites[blockIdx.x];
  const int blk = site_blk[site];
  if (threadIdx.x == 0) alpha_s = block_alpha<T>(part, blk_sites + (size_t)blk * bs, bs);
  __syncthreads();
  const int i = threadIdx.x;
  if (i < d) {
    const size_t o = (size_t)site * d + i;
    C<T> zz = z[o];
    cfma(zz, alpha_s, rho[o]);
    z[o] = zz;
  }
}

template <typename T, typename S>
void coarse_sap_colour(const CoarseOpView<T, S>& op, const int* blk_sites, const int* site_blk, int nblk,
                       int bs, int colour, int mr_iters, const C<T>* b, C<T>* z, SapScratch<T>& ws,
                       hipStream_t s) {
  if (mr_iters <= 0) return;
  DD_REQUIRE(op.d <= 64, "coarse levels support at most 64 components per site");
  const int nsites = (nblk / 2) * bs;
  const int* csites = blk_sites + (size_t)colour * (nblk / 2) * bs;   // blocks are colour-major
  with_nch(op.d, [&](auto nch) {
    constexpr int NCH = decltype(nch)::value;
    // the residual is rho_0 and lands in the "previous" buffer of step 0
    k_sap_res<T, S, NCH><<<nsites, 64 * SW, 0, s>>>(op, csites, b, z, ws.rho[1]);
    for (int t = 0; t < mr_iters; ++t) {
      const int pp = (t + 1) & 1, cc = t & 1;   // previous / current buffers
      k_sap_q<T, S, NCH><<<nsites, 64 * SW, 0, s>>>(op, csites, blk_sites, site_blk, bs, t, ws.rho[pp], ws.q[pp],
                                                ws.part[pp], ws.rho[cc], ws.q[cc], ws.part[cc], z);
    }
  });
  const int last = (mr_iters - 1) & 1;
  k_sap_fin<T><<<nsites, 64 * ((op.d + 63) / 64), 0, s>>>(op.d, csites, blk_sites, site_blk, bs,
                                                         ws.rho[last], ws.part[last], z);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// odd-even building blocks (site workgroups, as above)
// ---------------------------------------------------------------------------
template <typename T, typename S, int NCH>
__global__ void __launch_bounds__(64 * SW) k_csites(CoarseOpView<T, S> op, const int* __restrict__ sites,
                                                    T gamma, const C<T>* __restrict__ in_c, T alpha,
                                                    const C<T>* __restrict__ in_s, T beta,
                                                    const C<T>* __restrict__ in_h, C<T>* __restrict__ out) {
  __shared__ C<T> vin[9][64];
  __shared__ C<T> prow[SW][64];
  const int site = sites[blockIdx.x], w = threadIdx.x >> 6, lane = threadIdx.x & 63, d = op.d;
  unsigned mask = 0;
  if (alpha != T(0)) mask |= 1u;
  if (beta != T(0)) mask |= 0x1FEu;
  for (int e = threadIdx.x; e < 9 * d; e += blockDim.x) {
    const int k = e / d, j = e % d;
    if ((mask >> k) & 1u) {
      const C<T> v = (k == 0 ? in_s : in_h)[(size_t)op.nbr9[site * 9 + k] * d + j];
      vin[k][j] = k == 0 ? cscale(v, alpha) : cscale(v, beta);
    }
  }
  __syncthreads();
  const size_t bsz = (size_t)d * d;
  const C<T> r = site_rows_sum<T>(site_cols<T, S, NCH>(op.K + (size_t)site * 9 * bsz, bsz, vin, mask,
                                                     w * NCH, lane, d), prow);
  if (w == 0 && lane < d) {
    C<T> acc = r;
    if (gamma != T(0)) acc = cadd(acc, cscale(in_c[(size_t)site * d + lane], gamma));
    out[(size_t)site * d + lane] = acc;
  }
}

template <typename T, typename S>
void coarse_site_apply(const CoarseOpView<T, S>& op, const int* sites, int nsites, T gamma,
                       const C<T>* in_c, T alpha, const C<T>* in_s, T beta, const C<T>* in_h,
                       C<T>* out, hipStream_t s) {
  with_nch(op.d, [&](auto nch) {
    k_csites<T, S, decltype(nch)::value><<<nsites, 64 * SW, 0, s>>>(op, sites, gamma, in_c, alpha, in_s, beta,
                                                                 in_h, out);
  });
  DD_LAUNCH_CHECK();
}

template <typename T, int NCH>
__global__ void __launch_bounds__(64 * SW) k_site_matvec(const C<T>* __restrict__ M,
                                                         const int* __restrict__ sites, int d,
                                                         const C<T>* __restrict__ in, C<T>* __restrict__ out) {
  __shared__ C<T> vin[9][64];
  __shared__ C<T> prow[SW][64];
  const int k = blockIdx.x, site = sites[k], w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int e = threadIdx.x; e < d; e += blockDim.x) vin[0][e] = in[(size_t)site * d + e];
  __syncthreads();
  const C<T> r = site_rows_sum<T>(site_cols<T, C<T>, NCH>(M + (size_t)k * d * d, (size_t)d * d, vin, 1u,
                                                     w * NCH, lane, d), prow);
  if (w == 0 && lane < d) out[(size_t)site * d + lane] = r;
}

template <typename T>
void site_matvec(const C<T>* M, const int* sites, int nsites, int d, const C<T>* in, C<T>* out,
                 hipStream_t s) {
  with_nch(d, [&](auto nch) {
    k_site_matvec<T, decltype(nch)::value><<<nsites, 64 * SW, 0, s>>>(M, sites, d, in, out);
  });
  DD_LAUNCH_CHECK();
}

// Gauss-Jordan inversion of the self block of every listed site, FP64.
__global__ void k_self_inverse(const double2* __restrict__ D5, const int* __restrict__ sites, int d,
                               double2* __restrict__ inv) {
  extern __shared__ unsigned char smem_raw[];
  double2* a = reinterpret_cast<double2*>(smem_raw);     // [d][2d]
  __shared__ int piv;
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
    const double2 pinv = mk<double>(p.x / pn, -p.y / pn);
    __syncthreads();
    for (int c = threadIdx.x; c < w; c += blockDim.x) a[col * w + c] = cmul(a[col * w + c], pinv);
    __syncthreads();
    for (int e = threadIdx.x; e < d * w; e += blockDim.x) {
      const int r = e / w, c = e % w;
      if (r != col) {
        const double2 f = a[r * w + col];
        a[e] = csub(a[e], cmul(f, a[col * w + c]));
      }
    }
    __syncthreads();
  }
  // column-major result: element (r, c) at c*d + r
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int c = e / d, r = e % d;
    inv[(size_t)k * d * d + e] = a[r * w + d + c];
  }
}

void self_block_inverse(const double2* D, const int* sites, int nsites, int d, double2* inv,
                        hipStream_t s) {
  const size_t sm = (size_t)d * 2 * d * sizeof(double2);
  DD_CHECK_HIP(hipFuncSetAttribute((const void*)k_self_inverse,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm));
  k_self_inverse<<<nsites, 256, sm, s>>>(D, sites, d, inv);
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

#define DD_INST(T, S)                                                                            \
  template void coarse_apply<T, S>(const CoarseOpView<T, S>&, const C<T>*, C<T>*, hipStream_t);  \
  template void coarse_sap_colour<T, S>(const CoarseOpView<T, S>&, const int*, const int*, int, int, \
                                        int, int, const C<T>*, C<T>*, SapScratch<T>&, hipStream_t); \
  template void coarse_site_apply<T, S>(const CoarseOpView<T, S>&, const int*, int, T, const C<T>*, T, \
                                        const C<T>*, T, const C<T>*, C<T>*, hipStream_t);
DD_INST(double, double2)
DD_INST(float, float2)
DD_INST(float, __half2)
#undef DD_INST
template void site_matvec<double>(const double2*, const int*, int, int, const double2*, double2*, hipStream_t);
template void site_matvec<float>(const float2*, const int*, int, int, const float2*, float2*, hipStream_t);

}  // namespace ddamg
