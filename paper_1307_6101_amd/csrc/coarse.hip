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
  g.nbr.resize((size_t)g.V * 8);
  g.bipartite = true;
  for (int mu = 0; mu < 4; ++mu) g.bipartite = g.bipartite && (dims[mu] % 2 == 0);
  for (int s = 0; s < g.V; ++s) {
    int c[4], r = s;
    for (int mu = 0; mu < 4; ++mu) { c[mu] = r % dims[mu]; r /= dims[mu]; }
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[mu] = (cc[mu] + (dir == 0 ? 1 : dims[mu] - 1)) % dims[mu];
        g.nbr[s * 8 + 2 * mu + dir] = idx(cc);
      }
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
    g.site_loc.resize(g.V);
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
          g.site_loc[site] = l;
        }
        ++nbk;
      }
  }
  return g;
}

template <typename T>
__global__ void k_coarse_apply(CoarseOpView<T> op, const C<T>* __restrict__ in, C<T>* __restrict__ out) {
  const int site = blockIdx.x, i = threadIdx.x;
  if (i >= op.d) return;
  out[(size_t)site * op.d + i] = stencil_row<T>(op, in, site, i);
}

template <typename T>
void coarse_apply(const CoarseOpView<T>& op, const C<T>* in, C<T>* out, hipStream_t s) {
  const int bs = 64 * ((op.d + 63) / 64);
  k_coarse_apply<T><<<op.V, bs, 0, s>>>(op, in, out);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// coarse SAP colour pass: one workgroup per block, one thread per (site, row)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_coarse_sap(CoarseOpView<T> op, const int* __restrict__ blk_sites,
                             const int* __restrict__ site_blk, const int* __restrict__ site_loc,
                             int blk0, int bs, int mr_iters, const C<T>* __restrict__ b,
                             C<T>* __restrict__ z) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* rs = reinterpret_cast<C<T>*>(smem_raw);
  T* red = reinterpret_cast<T*>(rs + (size_t)bs * op.d);
  const int d = op.d;
  const int blk = blk0 + blockIdx.x;
  const int t = threadIdx.x;
  const bool valid = t < bs * d;
  const int sl = valid ? t / d : 0, i = valid ? t % d : 0;
  const int site = blk_sites[(size_t)blk * bs + sl];
  const size_t bsz = (size_t)d * d;
  C<T> rho = czero<T>(), x = czero<T>();
  if (valid) rho = csub(b[(size_t)site * d + i], stencil_row<T>(op, z, site, i));
  // in-block neighbours of this site
  int nloc[8];
  for (int k = 0; k < 8; ++k) {
    const int n = op.nbr[site * 8 + k];
    nloc[k] = site_blk[n] == blk ? site_loc[n] : -1;
  }
  const C<T>* Ds = op.D + (size_t)site * 5 * bsz;
  for (int it = 0; it < mr_iters; ++it) {
    if (valid) rs[t] = rho;
    __syncthreads();
    C<T> q = czero<T>();
    if (valid) {
      q = row_fwd<T>(Ds, rs + (size_t)sl * d, i, d);
      for (int mu = 0; mu < 4; ++mu) {
        if (nloc[2 * mu] >= 0)
          q = cadd(q, row_fwd<T>(Ds + (1 + mu) * bsz, rs + (size_t)nloc[2 * mu] * d, i, d));
        if (nloc[2 * mu + 1] >= 0) {
          const int nb = op.nbr[site * 8 + 2 * mu + 1];
          q = cadd(q, row_bwd<T>(op.D + ((size_t)nb * 5 + 1 + mu) * bsz,
                                 rs + (size_t)nloc[2 * mu + 1] * d, i, d));
        }
      }
    }
    T v[3] = {q.x * rho.x + q.y * rho.y, q.x * rho.y - q.y * rho.x, q.x * q.x + q.y * q.y};
    wg_sum<T, 3>(v, red);
    C<T> alpha = v[2] > T(0) ? mk<T>(v[0] / v[2], v[1] / v[2]) : czero<T>();
    cfma(x, alpha, rho);
    rho = csub(rho, cmul(alpha, q));
  }
  if (valid) z[(size_t)site * d + i] = cadd(z[(size_t)site * d + i], x);
}

template <typename T>
void coarse_sap_colour(const CoarseOpView<T>& op, const int* blk_sites, const int* site_blk,
                       const int* site_loc, int nblk, int bs, int colour, int mr_iters,
                       const C<T>* b, C<T>* z, hipStream_t s) {
  const int rows = bs * op.d;
  DD_REQUIRE(rows <= 1024, "coarse SAP block too large for one workgroup");
  const int wg = 64 * ((rows + 63) / 64);
  const size_t sm = (size_t)rows * sizeof(C<T>) + 16 * 3 * sizeof(T);
  k_coarse_sap<T><<<nblk / 2, wg, sm, s>>>(op, blk_sites, site_blk, site_loc, colour * (nblk / 2),
                                           bs, mr_iters, b, z);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// odd-even building blocks
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_site_apply(CoarseOpView<T> op, const int* __restrict__ sites, T gamma,
                             const C<T>* __restrict__ in_c, T alpha, const C<T>* __restrict__ in_s,
                             T beta, const C<T>* __restrict__ in_h, C<T>* __restrict__ out) {
  const int site = sites[blockIdx.x], i = threadIdx.x;
  const int d = op.d;
  if (i >= d) return;
  const size_t bsz = (size_t)d * d;
  const C<T>* Ds = op.D + (size_t)site * 5 * bsz;
  C<T> acc = czero<T>();
  if (gamma != T(0)) acc = cscale(in_c[(size_t)site * d + i], gamma);
  if (alpha != T(0)) acc = cadd(acc, cscale(row_fwd<T>(Ds, in_s + (size_t)site * d, i, d), alpha));
  if (beta != T(0)) {
    C<T> h = czero<T>();
    for (int mu = 0; mu < 4; ++mu) {
      const int nf = op.nbr[site * 8 + 2 * mu];
      h = cadd(h, row_fwd<T>(Ds + (1 + mu) * bsz, in_h + (size_t)nf * d, i, d));
      const int nb = op.nbr[site * 8 + 2 * mu + 1];
      h = cadd(h, row_bwd<T>(op.D + ((size_t)nb * 5 + 1 + mu) * bsz, in_h + (size_t)nb * d, i, d));
    }
    acc = cadd(acc, cscale(h, beta));
  }
  out[(size_t)site * d + i] = acc;
}

template <typename T>
void coarse_site_apply(const CoarseOpView<T>& op, const int* sites, int nsites, T gamma,
                       const C<T>* in_c, T alpha, const C<T>* in_s, T beta, const C<T>* in_h,
                       C<T>* out, hipStream_t s) {
  const int bs = 64 * ((op.d + 63) / 64);
  k_site_apply<T><<<nsites, bs, 0, s>>>(op, sites, gamma, in_c, alpha, in_s, beta, in_h, out);
  DD_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_site_matvec(const C<T>* __restrict__ M, const int* __restrict__ sites, int d,
                              const C<T>* __restrict__ in, C<T>* __restrict__ out) {
  const int k = blockIdx.x, site = sites[k], i = threadIdx.x;
  if (i >= d) return;
  out[(size_t)site * d + i] = row_fwd<T>(M + (size_t)k * d * d, in + (size_t)site * d, i, d);
}

template <typename T>
void site_matvec(const C<T>* M, const int* sites, int nsites, int d, const C<T>* in, C<T>* out,
                 hipStream_t s) {
  const int bs = 64 * ((d + 63) / 64);
  k_site_matvec<T><<<nsites, bs, 0, s>>>(M, sites, d, in, out);
  DD_LAUNCH_CHECK();
}

// Gauss-Jordan inversion of the self block of every listed site, FP64.
__global__ void k_self_inverse(const double2* __restrict__ D, const int* __restrict__ sites, int d,
                               double2* __restrict__ inv) {
  extern __shared__ unsigned char smem_raw[];
  double2* a = reinterpret_cast<double2*>(smem_raw);     // [d][2d]
  __shared__ int piv;
  const int k = blockIdx.x, site = sites[k];
  const int w = 2 * d;
  const double2* S = D + (size_t)site * 5 * d * d;
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
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int r = e / d, c = e % d;
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

// canonical export: [V][9][d][d] with blocks self, +mu (mu=0..3), -mu
__global__ void k_export_coarse(CoarseOpView<double> op, double2* __restrict__ out) {
  const int site = blockIdx.x, k = blockIdx.y;
  const int d = op.d, h = d / 2;
  const size_t bsz = (size_t)d * d;
  double2* o = out + ((size_t)site * 9 + k) * bsz;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int i = e / d, j = e % d;
    if (k < 5) {
      o[e] = op.D[((size_t)site * 5 + k) * bsz + e];
    } else {
      const int mu = k - 5;
      const int nb = op.nbr[site * 8 + 2 * mu + 1];
      const double2 f = op.D[((size_t)nb * 5 + 1 + mu) * bsz + (size_t)j * d + i];
      const double2 v = cconj(f);
      o[e] = ((i < h) == (j < h)) ? v : mk<double>(-v.x, -v.y);
    }
  }
}

void export_coarse(const CoarseOpView<double>& op, double2* out, hipStream_t s) {
  dim3 grid(op.V, 9);
  k_export_coarse<<<grid, 256, 0, s>>>(op, out);
  DD_LAUNCH_CHECK();
}

#define DD_INST(T)                                                                              \
  template void coarse_apply<T>(const CoarseOpView<T>&, const C<T>*, C<T>*, hipStream_t);      \
  template void coarse_sap_colour<T>(const CoarseOpView<T>&, const int*, const int*, const int*, \
                                     int, int, int, int, const C<T>*, C<T>*, hipStream_t);      \
  template void coarse_site_apply<T>(const CoarseOpView<T>&, const int*, int, T, const C<T>*, T, \
                                     const C<T>*, T, const C<T>*, C<T>*, hipStream_t);          \
  template void site_matvec<T>(const C<T>*, const int*, int, int, const C<T>*, C<T>*, hipStream_t);
DD_INST(double)
DD_INST(float)
#undef DD_INST

}  // namespace ddamg
