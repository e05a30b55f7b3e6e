// Fine-lattice kernels: layout conversion, clover construction, the
// Wilson-clover stencil and the red-black SAP colour pass with block MR.
//
// Operator (the paper's eq. (1); definition of D as in the two-level
// predecessor, textbook Sheikholeslami-Wohlert form):
//   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu)
//                                         + (1+g_mu) U_mu(x-mu)^H psi(x-mu) ]
//   A(x) = (m0+4) - c_sw/16 sum_{mu<nu} g_mu g_nu (x) (Q_mu,nu - Q_mu,nu^H),
// chiral gamma basis, Gamma5 = diag(1,1,-1,-1): A(x) is block diagonal with
// one Hermitian 6x6 block per chirality.
//
// Spin projection.  With g_mu = [[0, B_mu],[B_mu^H, 0]], (1 -+ g_mu) psi is
// fixed by its upper half h = (psi_0 + c0 psi_j0, psi_1 + c1 psi_j1), with
// (j0, c0, j1, c1) = (3, i, 2, i), (3, 1, 2, -1), (2, i, 3, -i), (2, -1, 3, -1)
// for mu = 0..3 in the forward hop and c -> -c in the backward hop; the lower
// half is rebuilt as out_j0 += conj(c0) chi_0, out_j1 += conj(c1) chi_1 with
// chi = U h.  So each hop moves 6 instead of 12 complex numbers through the
// SU(3) multiply.
#include "fine.h"
#include "fine_dev.h"

#include <type_traits>

#include <vector>

namespace ddamg {

FineGeom make_fine_geom(const int dims[4]) {
  FineGeom g;
  g.V = 1;
  g.nblk = 1;
  for (int mu = 0; mu < 4; ++mu) {
    DD_REQUIRE(dims[mu] % 4 == 0, "every lattice extent must be a multiple of 4");
    g.dims[mu] = dims[mu];
    g.nb[mu] = dims[mu] / 2;
    g.V *= dims[mu];
    g.nblk *= g.nb[mu];
  }
  return g;
}

void fine_tables(const FineGeom& g, int* nbr_blk, int* colour_blocks) {
  int n[2] = {0, 0};
  const int half = g.nblk / 2;
  for (int b = 0; b < g.nblk; ++b) {
    int c[4];
    block_decode(g.nb, b, c);
    for (int mu = 0; mu < 4; ++mu) {
      for (int dir = 0; dir < 2; ++dir) {
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[mu] = (cc[mu] + (dir == 0 ? 1 : g.nb[mu] - 1)) % g.nb[mu];
        nbr_blk[b * 8 + 2 * mu + dir] = block_encode(g.nb, cc);
      }
    }
    int col = (c[0] + c[1] + c[2] + c[3]) & 1;
    colour_blocks[col * half + n[col]++] = b;
  }
}

// ---------------------------------------------------------------------------
// index helpers
// ---------------------------------------------------------------------------
struct DevGeom {
  int X, Y, Z, T;
  int nb[4];
  long long V;
};
static DevGeom devgeom(const FineGeom& g) {
  return DevGeom{g.dims[0], g.dims[1], g.dims[2], g.dims[3], {g.nb[0], g.nb[1], g.nb[2], g.nb[3]}, g.V};
}

__device__ inline void canonical_to_native(const DevGeom& g, long long i, int& blk, int& loc) {
  int x = (int)(i % g.X);
  long long r = i / g.X;
  int y = (int)(r % g.Y);
  r /= g.Y;
  int z = (int)(r % g.Z);
  int t = (int)(r / g.Z);
  const int b[4] = {x >> 1, y >> 1, z >> 1, t >> 1};
  blk = block_encode(g.nb, b);
  loc = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((t & 1) << 3);
}

__device__ inline long long canon_index(const DevGeom& g, int x, int y, int z, int t) {
  x = (x + g.X) % g.X;
  y = (y + g.Y) % g.Y;
  z = (z + g.Z) % g.Z;
  t = (t + g.T) % g.T;
  return x + (long long)g.X * (y + (long long)g.Y * (z + (long long)g.Z * t));
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_to_native(DevGeom g, const double2* __restrict__ in, C<T>* __restrict__ out) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const long long off = (long long)blockIdx.y * g.V * 12;
  int blk, loc;
  canonical_to_native(g, i, blk, loc);
#pragma unroll
  for (int c = 0; c < 12; ++c)
    out[off + ((long long)blk * 12 + c) * 16 + loc] = ccast<T>(in[off + i * 12 + c]);
}

template <typename T>
__global__ void k_from_native(DevGeom g, const C<T>* __restrict__ in, double2* __restrict__ out) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const long long off = (long long)blockIdx.y * g.V * 12;
  int blk, loc;
  canonical_to_native(g, i, blk, loc);
#pragma unroll
  for (int c = 0; c < 12; ++c)
    out[off + i * 12 + c] = ccast<double>(in[off + ((long long)blk * 12 + c) * 16 + loc]);
}

template <typename T>
__global__ void k_links_to_native(DevGeom g, const double2* __restrict__ in, C<T>* __restrict__ out) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  int blk, loc;
  canonical_to_native(g, i, blk, loc);
  for (int e = 0; e < 36; ++e)
    out[((long long)blk * 36 + e) * 16 + loc] = ccast<T>(in[i * 36 + e]);
}

template <typename T>
void fine_to_native(const FineGeom& g, const double2* in, C<T>* out, int nrhs, hipStream_t s) {
  dim3 grid(nblocks(g.V, 256), nrhs);
  k_to_native<T><<<grid, 256, 0, s>>>(devgeom(g), in, out);
  DD_LAUNCH_CHECK();
}
template <typename T>
void fine_from_native(const FineGeom& g, const C<T>* in, double2* out, int nrhs, hipStream_t s) {
  dim3 grid(nblocks(g.V, 256), nrhs);
  k_from_native<T><<<grid, 256, 0, s>>>(devgeom(g), in, out);
  DD_LAUNCH_CHECK();
}
template <typename T>
void links_to_native(const FineGeom& g, const double2* links, C<T>* out, hipStream_t s) {
  k_links_to_native<T><<<nblocks(g.V, 256), 256, 0, s>>>(devgeom(g), links, out);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// clover construction (FP64, canonical links in, native packed out)
// ---------------------------------------------------------------------------
struct M3 { double2 e[9]; };

__device__ inline M3 load_link(const double2* L, long long site, int mu) {
  M3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) m.e[k] = L[(site * 4 + mu) * 9 + k];
  return m;
}
// a * b, a^H * b, a * b^H
__device__ inline M3 mm(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = czero<double>();
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(s, a.e[i * 3 + k], b.e[k * 3 + j]);
      c.e[i * 3 + j] = s;
    }
  return c;
}
__device__ inline M3 mhm(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = czero<double>();
#pragma unroll
      for (int k = 0; k < 3; ++k) cjfma(s, a.e[k * 3 + i], b.e[k * 3 + j]);
      c.e[i * 3 + j] = s;
    }
  return c;
}
__device__ inline M3 mmh(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = czero<double>();
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(s, a.e[i * 3 + k], cconj(b.e[j * 3 + k]));
      c.e[i * 3 + j] = s;
    }
  return c;
}

// chiral-basis gamma matrices, entries as (re, im)
__constant__ double c_gamma[4][4][4][2] = {
    {{{0, 0}, {0, 0}, {0, 0}, {0, -1}}, {{0, 0}, {0, 0}, {0, -1}, {0, 0}},
     {{0, 0}, {0, 1}, {0, 0}, {0, 0}}, {{0, 1}, {0, 0}, {0, 0}, {0, 0}}},
    {{{0, 0}, {0, 0}, {0, 0}, {-1, 0}}, {{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}}, {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},
    {{{0, 0}, {0, 0}, {0, -1}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}, {0, 1}},
     {{0, 1}, {0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {0, -1}, {0, 0}, {0, 0}}},
    {{{0, 0}, {0, 0}, {1, 0}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}, {1, 0}},
     {{1, 0}, {0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {1, 0}, {0, 0}, {0, 0}}}};

__device__ inline double2 gam(int mu, int a, int b) {
  return mk<double>(c_gamma[mu][a][b][0], c_gamma[mu][a][b][1]);
}

__global__ void k_clover(DevGeom g, const double2* __restrict__ L, double m0, double csw,
                         double2* __restrict__ out) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  int xc[4];
  {
    long long r = i;
    xc[0] = (int)(r % g.X); r /= g.X;
    xc[1] = (int)(r % g.Y); r /= g.Y;
    xc[2] = (int)(r % g.Z); xc[3] = (int)(r / g.Z);
  }
  auto nbr = [&](int mu, int smu, int nu, int snu) {
    int c[4] = {xc[0], xc[1], xc[2], xc[3]};
    c[mu] += smu;
    c[nu] += snu;
    return canon_index(g, c[0], c[1], c[2], c[3]);
  };
  // A_chi[6][6], chi = 0 (spins 0,1), 1 (spins 2,3)
  double2 A[2][6][6];
  for (int h = 0; h < 2; ++h)
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) A[h][a][b] = czero<double>();
  if (csw != 0.0) {
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        M3 Um = load_link(L, i, mu), Un = load_link(L, i, nu);
        M3 Um_pn = load_link(L, nbr(nu, 1, mu, 0), mu);      // U_mu(x+nu)
        M3 Un_pm = load_link(L, nbr(mu, 1, nu, 0), nu);      // U_nu(x+mu)
        M3 Um_mm = load_link(L, nbr(mu, -1, nu, 0), mu);     // U_mu(x-mu)
        M3 Un_mm = load_link(L, nbr(mu, -1, nu, 0), nu);     // U_nu(x-mu)
        M3 Um_pnmm = load_link(L, nbr(mu, -1, nu, 1), mu);   // U_mu(x+nu-mu)
        M3 Um_mmmn = load_link(L, nbr(mu, -1, nu, -1), mu);  // U_mu(x-mu-nu)
        M3 Un_mmmn = load_link(L, nbr(mu, -1, nu, -1), nu);  // U_nu(x-mu-nu)
        M3 Um_mn = load_link(L, nbr(nu, -1, mu, 0), mu);     // U_mu(x-nu)
        M3 Un_mn = load_link(L, nbr(nu, -1, mu, 0), nu);     // U_nu(x-nu)
        M3 Un_mnpm = load_link(L, nbr(mu, 1, nu, -1), nu);   // U_nu(x-nu+mu)
        // four counter-clockwise leaves at x
        M3 q1 = mmh(mmh(mm(Um, Un_pm), Um_pn), Un);
        // Un(x) Um(x+nu-mu)^H Un(x-mu)^H Um(x-mu)
        M3 q2 = mm(mmh(mmh(Un, Um_pnmm), Un_mm), Um_mm);
        // leaf 3: Um(x-mu)^H Un(x-mu-nu)^H Um(x-mu-nu) Un(x-nu)
        M3 t3 = mhm(Un_mmmn, mm(Um_mmmn, Un_mn));           // Un(x-mu-nu)^H Um(x-mu-nu) Un(x-nu)
        M3 l3 = mhm(Um_mm, t3);
        // leaf 4: Un(x-nu)^H Um(x-nu) Un(x-nu+mu) Um(x)^H
        M3 l4 = mmh(mhm(Un_mn, mm(Um_mn, Un_mnpm)), Um);
        M3 F;
#pragma unroll
        for (int k = 0; k < 9; ++k) F.e[k] = cadd(cadd(q1.e[k], q2.e[k]), cadd(l3.e[k], l4.e[k]));
        // F <- Q - Q^H
        M3 Fa;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) Fa.e[a * 3 + b] = csub(F.e[a * 3 + b], cconj(F.e[b * 3 + a]));
        // sigma = g_mu g_nu (block diagonal in chirality)
        for (int h = 0; h < 2; ++h)
          for (int s = 0; s < 2; ++s)
            for (int sp = 0; sp < 2; ++sp) {
              double2 sg = czero<double>();
              for (int k = 0; k < 4; ++k) cfma(sg, gam(mu, 2 * h + s, k), gam(nu, k, 2 * h + sp));
              sg = cscale(sg, -csw / 16.0);
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) cfma(A[h][s * 3 + a][sp * 3 + b], sg, Fa.e[a * 3 + b]);
            }
      }
  }
  int blk, loc;
  canonical_to_native(g, i, blk, loc);
  double2* o = out + (long long)blk * 36 * 16 + loc;
  for (int h = 0; h < 2; ++h) {
    double d[6];
    for (int a = 0; a < 6; ++a) d[a] = A[h][a][a].x + (m0 + 4.0);
    for (int k = 0; k < 3; ++k) o[(h * 18 + k) * 16] = mk<double>(d[2 * k], d[2 * k + 1]);
    int e = 3;
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b) o[(h * 18 + e++) * 16] = A[h][a][b];
  }
}

void clover_build(const FineGeom& g, const double2* links, double m0, double csw, double2* out,
                  hipStream_t s) {
  k_clover<<<nblocks(g.V, 128), 128, 0, s>>>(devgeom(g), links, m0, csw, out);
  DD_LAUNCH_CHECK();
}

// the eight neighbour blocks of `blk` (2*mu + 0: +mu, 2*mu + 1: -mu), two
// 16-byte loads issued together so that no later load waits on an index
struct Nbr8 {
  int v[8];
};
__device__ inline Nbr8 load_nbr8(const int* __restrict__ nbr, int blk) {
  const int4* p = reinterpret_cast<const int4*>(nbr + (size_t)blk * 8);
  const int4 a = p[0], b = p[1];
  return Nbr8{{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}};
}

// (the input field in spinor storage V: C<T>, or FP16 with site scales ins)
template <typename T, typename S, typename V, int MU>
__device__ inline void hops_mu(const FineOpView<T, S>& op, const V* __restrict__ in, const float* __restrict__ ins,
                               int blk, int loc, const Nbr8& nb8, C<T> acc[12]) {
  constexpr int bit = 1 << MU;
  C<T> psi[12], u[9];
  // forward: psi(x+mu), U_mu(x)
  {
    const int nb = (loc & bit) ? nb8.v[2 * MU] : blk;
    load_site<T, V>(in, ins, nb, loc ^ bit, psi);
    load_link<T, S>(op.U, blk, loc, MU, u);
    hop_apply<T, MU, true>(psi, u, acc);
  }
  // backward: psi(x-mu), U_mu(x-mu)^H
  {
    const int nb = (loc & bit) ? blk : nb8.v[2 * MU + 1];
    load_site<T, V>(in, ins, nb, loc ^ bit, psi);
    load_link<T, S>(op.U, nb, loc ^ bit, MU, u);
    hop_apply<T, MU, false>(psi, u, acc);
  }
}

// out(x) = (D in)(x) for one site
template <typename T, typename S, typename V = C<T>>
__device__ inline void dslash_site(const FineOpView<T, S>& op, const V* __restrict__ in,
                                   const float* __restrict__ ins, int blk, int loc, C<T> out[12]) {
  const Nbr8 nb8 = load_nbr8(op.nbr, blk);
  C<T> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = czero<T>();
  hops_mu<T, S, V, 0>(op, in, ins, blk, loc, nb8, acc);
  hops_mu<T, S, V, 1>(op, in, ins, blk, loc, nb8, acc);
  hops_mu<T, S, V, 2>(op, in, ins, blk, loc, nb8, acc);
  hops_mu<T, S, V, 3>(op, in, ins, blk, loc, nb8, acc);
  C<T> psi[12];
  load_site<T, V>(in, ins, blk, loc, psi);
  clover_apply<T, S>(op.A, blk, loc, psi, out);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    out[c].x -= T(0.5) * acc[c].x;
    out[c].y -= T(0.5) * acc[c].y;
  }
}

// One site per thread.  A batch of nb fields runs over a one-dimensional
// grid of gx * nb workgroups with the XCD-aware batch mapping.
template <typename T, typename S, typename V = C<T>>
__global__ void __launch_bounds__(256) k_dslash(FineOpView<T, S> op, const V* __restrict__ in,
                                                const float* __restrict__ ins, C<T>* __restrict__ out,
                                                long long fs, int gx, int nb) {
  int x, r;
  xcd_slab_rhs(blockIdx.x, gx, nb, x, r);
  const int tid = x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15;
  if (blk >= op.nblk) return;
  in += (long long)r * fs;
  if constexpr (std::is_same<V, __half2>::value) ins += (long long)r * (fs / 12);
  out += (long long)r * fs;
  C<T> o[12];
  dslash_site<T, S, V>(op, in, ins, blk, loc, o);
  C<T>* p = out + (long long)blk * 192 + loc;
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c * 16] = o[c];
}

template <typename T, typename S>
void dslash(const FineOpView<T, S>& op, const C<T>* in, C<T>* out, hipStream_t s, int nb) {
  const long long fs = (long long)op.nblk * 192;
  const unsigned gx = nblocks((size_t)op.nblk * 16, 256);
  k_dslash<T, S><<<gx * nb, 256, 0, s>>>(op, in, nullptr, out, fs, (int)gx, nb);
  DD_LAUNCH_CHECK();
}

void dslash_hs(const FineOpView<double>& op, const __half2* in, const float* ins, double2* out, hipStream_t s,
               int nb) {
  const long long fs = (long long)op.nblk * 192;
  const unsigned gx = nblocks((size_t)op.nblk * 16, 256);
  k_dslash<double, double2, __half2><<<gx * nb, 256, 0, s>>>(op, in, ins, out, fs, (int)gx, nb);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// SAP colour pass.  One thread per site, 16 lanes per 2^4 block, 16 blocks
// per workgroup; a batch of fields runs one field per workgroup with the
// XCD-aware batch mapping.  r = b - D z with the full operator (the blocks'
// z staged in LDS: the in-block neighbours come from there, the others from
// memory), then mr_iters minimal residual steps on the Dirichlet block
// operator D_i (self term + the four in-block hops, partner spinors
// exchanged through LDS, block sums of the step sizes by DPP row moves),
// z += x.  The four in-block links of a site are read once into registers,
// in their stored precision and as the site applies them (U for the lower
// site of a pair, U^H for the upper one), so that forward and backward
// in-block hops run the same instructions; with FP16 storage the clover is
// kept in LDS for the pass.
// ---------------------------------------------------------------------------
// The in-block hop of direction MU: forward (the lower site of the pair,
// link U) or backward (the upper site, U^H), with the link passed as the site
// applies it; the backward hop's projection phases are the forward ones times
// -1 (sg), so every lane runs the same instructions.
template <typename T, int MU, typename G>
__device__ inline void oriented_hop(G&& get, T sg, const C<T> (&u)[9], C<T> acc[12]) {
  using P = Proj<MU>;
  constexpr int c0 = (4 - P::K0) & 3, c1 = (4 - P::K1) & 3;
  C<T> h[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const C<T> p0 = get(a), p1 = get(3 + a);
    const C<T> q0 = mul_ik<P::K0>(get(P::J0 * 3 + a));
    const C<T> q1 = mul_ik<P::K1>(get(P::J1 * 3 + a));
    h[a] = mk<T>(fma(sg, q0.x, p0.x), fma(sg, q0.y, p0.y));
    h[3 + a] = mk<T>(fma(sg, q1.x, p1.x), fma(sg, q1.y, p1.y));
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C<T> v = cmul(u[a * 3], h[s * 3]);
      cfma(v, u[a * 3 + 1], h[s * 3 + 1]);
      cfma(v, u[a * 3 + 2], h[s * 3 + 2]);
      acc[s * 3 + a] = cadd(acc[s * 3 + a], v);
      const int j = s ? P::J1 : P::J0;
      const C<T> w = s ? mul_ik<c1>(v) : mul_ik<c0>(v);
      acc[j * 3 + a] = mk<T>(fma(sg, w.x, acc[j * 3 + a].x), fma(sg, w.y, acc[j * 3 + a].y));
    }
}

// The in-block hop of direction MU, the neighbour's spinor in LDS (rs,
// [12][256], the site at column t): forward for the lower site of the pair,
// backward for the upper one
template <typename T, typename S, int MU>
__device__ inline void inblock_hop(const C<T>* __restrict__ rs, int t, int loc, const C<T> (&u)[9],
                                   C<T> acc[12]) {
  constexpr int bit = 1 << MU;
  const T sg = (loc & bit) ? T(-1) : T(1);
  oriented_hop<T, MU>([&](int c) { return rs[c * 256 + (t ^ bit)]; }, sg, u, acc);
}

// The site's in-block links: loaded into registers once per pass for the
// residual's in-block hops and the MR steps (FP32 and FP16 storage) or read
// again at every use (FP64, where registers do not suffice).  The clover is read at every step: keeping it too (144 more
// registers in FP32) leaves one wavefront per SIMD and was measured slower.
// The link of in-block direction mu as the site applies it: the link
// joining loc and loc ^ (1 << mu) belongs to the lower site, which applies
// U; the upper site applies U^H (the transposed entries, conjugated).
template <typename T, typename S>
__device__ inline void oriented_link(const S* __restrict__ U, int blk, int loc, int mu, C<T> (&u)[9]) {
  const bool up = (loc >> mu) & 1;
  const S* p = U + (long long)blk * 576 + mu * 144 + (loc & ~(1 << mu));
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const C<T> v = ldc<T, S>(p[(up ? b * 3 + a : a * 3 + b) * 16]);
      u[a * 3 + b] = up ? cconj(v) : v;
    }
}

template <typename T, typename S, bool KEEP> struct BlockOp {
  S ul[KEEP ? 4 : 1][9];
  __device__ void load(const FineOpView<T, S>& op, int blk, int loc, bool valid) {
    if constexpr (KEEP) {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        const bool up = (loc >> mu) & 1;
        const S* p = op.U + (long long)blk * 576 + mu * 144 + (loc & ~(1 << mu));
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            S v = p[(up ? b * 3 + a : a * 3 + b) * 16];
            if (up) v.y = -v.y;
            ul[mu][a * 3 + b] = v;
          }
      }
    }
  }
  // the link as this site applies it (U or U^H)
  __device__ void link(const FineOpView<T, S>& op, int blk, int loc, int mu, C<T> (&u)[9]) const {
    if constexpr (KEEP) {
#pragma unroll
      for (int k = 0; k < 9; ++k) u[k] = ldc<T, S>(ul[mu][k]);
    } else {
      oriented_link<T, S>(op.U, blk, loc, mu, u);
    }
  }
  __device__ void clover(const FineOpView<T, S>& op, int blk, int loc, const C<T> v[12], C<T> out[12]) const {
    clover_apply<T, S>(op.A, blk, loc, v, out);
  }
};

// Whether a colour pass keeps each site's clover in LDS (one private slot
// per thread, [36][256] entries of the stored type) for its MR steps instead
// of reading it from memory at every step: for FP16 storage the slots take
// 36 KiB of a workgroup's LDS, which leaves the kernel's occupancy (set by
// its registers) unchanged; in FP32 they would take 72 KiB and halve it.
template <typename S> struct ClLds : std::false_type {};
template <> struct ClLds<__half2> : std::true_type {};

// Completes the arithmetic that produces acc before the statements that
// follow (empty asm statements that read and write it), so that the next
// direction's loads are not all issued ahead of it: hoisting the eight hops'
// loads would need more registers than the colour pass can hold at two
// wavefronts per SIMD.
template <typename T> __device__ inline void pin12(C<T> (&acc)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(acc[c].x), "+v"(acc[c].y));
}

// The out-of-block hop of direction MU in the residual of a SAP block site:
// the neighbour outside the block is x+mu for the upper site of the pair
// (link U_mu(x), the site's own) and x-mu for the lower one (link
// U_mu(x-mu) of the neighbour block's site, applied as U^H).  The link is
// loaded oriented, so both kinds of site run the same instructions.
template <typename T, typename S, typename V, int MU>
__device__ inline void sap_outer_hop(const FineOpView<T, S>& op, const V* __restrict__ in,
                                     const float* __restrict__ ins, int blk, int loc, const Nbr8& nb8,
                                     C<T> (&acc)[12]) {
  constexpr int bit = 1 << MU;
  const bool up = loc & bit;
  const int nbb = up ? nb8.v[2 * MU] : nb8.v[2 * MU + 1];
  C<T> psi[12], u[9];
  load_site<T, V>(in, ins, nbb, loc ^ bit, psi);
  const S* p = op.U + (long long)(up ? blk : nbb) * 576 + MU * 144 + (up ? loc : loc ^ bit);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const C<T> v = ldc<T, S>(p[(up ? a * 3 + b : b * 3 + a) * 16]);
      u[a * 3 + b] = up ? v : cconj(v);
    }
  oriented_hop<T, MU>([&](int c) { return psi[c]; }, up ? T(1) : T(-1), u, acc);
}

// Both hops of direction MU in the residual: the out-of-block one from
// memory, the in-block one from the staged z (rs) with the link the site
// keeps for its MR steps
template <typename T, typename S, typename V, int MU, typename B>
__device__ inline void sap_hops_mu(const FineOpView<T, S>& op, const V* __restrict__ in, const float* __restrict__ ins,
                                   const C<T>* rs, int t, int blk, int loc, const Nbr8& nb8, const B& bop,
                                   C<T> (&acc)[12]) {
  sap_outer_hop<T, S, V, MU>(op, in, ins, blk, loc, nb8, acc);
  C<T> u[9];
  bop.link(op, blk, loc, MU, u);
  inblock_hop<T, S, MU>(rs, t, loc, u, acc);
  pin12<T>(acc);
}

// a site's spinor from its stored components (and FP16 scale m), as load_site
template <typename T, typename V>
__device__ inline void decode_kept(const V (&raw)[12], float m, C<T> v[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    v[c] = ldc<T, V>(raw[c]);
    if constexpr (std::is_same<V, __half2>::value) {
      v[c].x *= T(m);
      v[c].y *= T(m);
    }
  }
}

// one workgroup per (chunk of 16 blocks, field of the batch), gx chunks;
// b and z in spinor storage V (bs, zs: their site scales for FP16)
template <typename T, typename S, typename V>
__global__ void __launch_bounds__(256) k_sap_colour(FineOpView<T, S> op, const int* __restrict__ cblk,
                                                    int ncb, int mr_iters, const V* __restrict__ b,
                                                    const float* __restrict__ bs, V* __restrict__ z,
                                                    float* __restrict__ zs, int nb, long long fs, int gx) {
  __shared__ C<T> rs[12 * 256];
  constexpr bool CL = ClLds<S>::value;
  __shared__ S cl[CL ? 36 * 256 : 1];
  const int t = threadIdx.x;
  int xw, rw;
  xcd_slab_rhs(blockIdx.x, gx, nb, xw, rw);
  b += (long long)rw * fs;
  z += (long long)rw * fs;
  constexpr bool HS = std::is_same<V, __half2>::value;
  if constexpr (HS) {
    bs += (long long)rw * (fs / 12);
    zs += (long long)rw * (fs / 12);
  }
  const int jb = xw * 16 + (t >> 4);
  const int loc = t & 15;
  const bool valid = jb < ncb;
  const int blk = valid ? cblk[jb] : 0;
  constexpr bool KEEP = !std::is_same<T, double>::value;
  BlockOp<T, S, KEEP> bop;
  {
    C<T> rho[12], x[12];
    if constexpr (CL) {
      // the site's clover into its private LDS slot (read once per pass)
      const S* pa = op.A + (long long)blk * 576 + loc;
#pragma unroll
      for (int e = 0; e < 36; ++e) cl[e * 256 + t] = pa[e * 16];
    }
    // the block's z in LDS: in-block neighbours and the site itself come
    // from there, the other neighbours from memory.  In FP32 arithmetic the
    // site's z also stays in registers as stored (and its scale) for the
    // final z += x
    constexpr bool KZ = !std::is_same<T, double>::value;
    V zkeep[KZ ? 12 : 1];
    float zsk = 1.f;
    {
      C<T> zz[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) zz[c] = czero<T>();
      if (valid) {
        if constexpr (KZ) {
          const V* pz = z + (long long)blk * 192 + loc;
#pragma unroll
          for (int c = 0; c < 12; ++c) zkeep[c] = pz[c * 16];
          if constexpr (HS) zsk = zs[(long long)blk * 16 + loc];
          decode_kept<T, V>(zkeep, zsk, zz);
        } else {
          load_site<T, V>(z, zs, blk, loc, zz);
        }
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) rs[c * 256 + t] = zz[c];
    }
    // the in-block links, for the residual's in-block hops and the MR steps
    bop.load(op, blk, loc, valid);
    __syncthreads();
    if (valid) {
      const Nbr8 nb8 = load_nbr8(op.nbr, blk);
      C<T> acc[12], zz[12], dz[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = czero<T>();
      sap_hops_mu<T, S, V, 0>(op, z, zs, rs, t, blk, loc, nb8, bop, acc);
      sap_hops_mu<T, S, V, 1>(op, z, zs, rs, t, blk, loc, nb8, bop, acc);
      sap_hops_mu<T, S, V, 2>(op, z, zs, rs, t, blk, loc, nb8, bop, acc);
      sap_hops_mu<T, S, V, 3>(op, z, zs, rs, t, blk, loc, nb8, bop, acc);
#pragma unroll
      for (int c = 0; c < 12; ++c) zz[c] = rs[c * 256 + t];
      if constexpr (CL) clover_mul<T>([&](int e) { return ldc<T, S>(cl[e * 256 + t]); }, zz, dz);
      else clover_apply<T, S>(op.A, blk, loc, zz, dz);
      C<T> bb[12];
      load_site<T, V>(b, bs, blk, loc, bb);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        rho[c].x = bb[c].x - dz[c].x + T(0.5) * acc[c].x;
        rho[c].y = bb[c].y - dz[c].y + T(0.5) * acc[c].y;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = czero<T>();
    }
    __syncthreads();   // rs is rewritten by the first MR step
#pragma unroll
    for (int c = 0; c < 12; ++c) x[c] = czero<T>();

    for (int it = 0; it < mr_iters; ++it) {
#pragma unroll
      for (int c = 0; c < 12; ++c) rs[c * 256 + t] = rho[c];
      __syncthreads();
      C<T> q[12], acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = czero<T>();
      {
        C<T> u[9];
        bop.link(op, blk, loc, 0, u);
        inblock_hop<T, S, 0>(rs, t, loc, u, acc);
        bop.link(op, blk, loc, 1, u);
        inblock_hop<T, S, 1>(rs, t, loc, u, acc);
        bop.link(op, blk, loc, 2, u);
        inblock_hop<T, S, 2>(rs, t, loc, u, acc);
        bop.link(op, blk, loc, 3, u);
        inblock_hop<T, S, 3>(rs, t, loc, u, acc);
      }
      if constexpr (CL) clover_mul<T>([&](int e) { return ldc<T, S>(cl[e * 256 + t]); }, rho, q);
      else bop.clover(op, blk, loc, rho, q);
      T qr_re = 0, qr_im = 0, qq = 0;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        q[c].x = rfma(T(-0.5), acc[c].x, q[c].x);
        q[c].y = rfma(T(-0.5), acc[c].y, q[c].y);
        qr_re = rfma(q[c].x, rho[c].x, qr_re);
        qr_re = rfma(q[c].y, rho[c].y, qr_re);
        qr_im = rfma(q[c].x, rho[c].y, qr_im);
        qr_im = rfma(-q[c].y, rho[c].x, qr_im);
        qq = rfma(q[c].x, q[c].x, qq);
        qq = rfma(q[c].y, q[c].y, qq);
      }
      qr_re = sum16<T>(qr_re);
      qr_im = sum16<T>(qr_im);
      qq = sum16<T>(qq);
      const T iq = qq > T(0) ? T(1) / qq : T(0);
      const C<T> alpha = mk<T>(qr_re * iq, qr_im * iq);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        cfma(x[c], alpha, rho[c]);
        cfma(rho[c], mk<T>(-alpha.x, -alpha.y), q[c]);
      }
      __syncthreads();
    }
    if (valid) {
      // z + x (for FP16 spinors re-encoded with the site's new scale)
      C<T> zz[12];
      if constexpr (KZ) decode_kept<T, V>(zkeep, zsk, zz);
      else load_site<T, V>(z, zs, blk, loc, zz);
#pragma unroll
      for (int c = 0; c < 12; ++c) zz[c] = cadd(zz[c], x[c]);
      store_site<T, V>(z, zs, blk, loc, zz);
    }
  }
}


template <typename T, typename S>
void sap_colour(const FineOpView<T, S>& op, const int* colour_blocks, int colour, int mr_iters,
                const C<T>* b, C<T>* z, hipStream_t s, int nb) {
  const int ncb = op.nblk / 2;
  const long long fs = (long long)op.nblk * 192;
  const unsigned gx = nblocks(ncb, 16);
  k_sap_colour<T, S, C<T>><<<gx * nb, 256, 0, s>>>(op, colour_blocks + colour * ncb, ncb, mr_iters, b, nullptr,
                                                   z, nullptr, nb, fs, (int)gx);
  DD_LAUNCH_CHECK();
}

void sap_colour_hs(const FineOpView<float, __half2>& op, const int* colour_blocks, int colour, int mr_iters,
                   const __half2* b, const float* bs, __half2* z, float* zs, hipStream_t s, int nb) {
  const int ncb = op.nblk / 2;
  const long long fs = (long long)op.nblk * 192;
  const unsigned gx = nblocks(ncb, 16);
  k_sap_colour<float, __half2, __half2><<<gx * nb, 256, 0, s>>>(op, colour_blocks + colour * ncb, ncb, mr_iters,
                                                                b, bs, z, zs, nb, fs, (int)gx);
  DD_LAUNCH_CHECK();
}

// explicit instantiations
#define DD_INST(T)                                                                              \
  template void fine_to_native<T>(const FineGeom&, const double2*, C<T>*, int, hipStream_t);   \
  template void fine_from_native<T>(const FineGeom&, const C<T>*, double2*, int, hipStream_t); \
  template void links_to_native<T>(const FineGeom&, const double2*, C<T>*, hipStream_t);       \
  template void dslash<T, C<T>>(const FineOpView<T, C<T>>&, const C<T>*, C<T>*, hipStream_t, int); \
  template void sap_colour<T, C<T>>(const FineOpView<T, C<T>>&, const int*, int, int, const C<T>*, \
                                    C<T>*, hipStream_t, int);
DD_INST(double)
DD_INST(float)
#undef DD_INST
template void dslash<float, __half2>(const FineOpView<float, __half2>&, const float2*, float2*, hipStream_t,
                                    int);
template void sap_colour<float, __half2>(const FineOpView<float, __half2>&, const int*, int, int, const float2*,
                                         float2*, hipStream_t, int);

__global__ void k_to_half(const double2* __restrict__ in, __half2* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = __floats2half2_rn((float)in[i].x, (float)in[i].y);
}

__global__ void k_gamma5(const double2* in, double2* out, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    // native layout [block][component][16 sites]: component (i / 16) % 12
    const int c = (int)((i >> 4) % 12);
    const double2 v = in[i];
    out[i] = c < 6 ? v : make_double2(-v.x, -v.y);
  }
}

void gamma5(const FineGeom& g, const double2* in, double2* out, int nb, hipStream_t s) {
  const long long n = (long long)g.nblk * 192 * nb;
  long long gr = (n + 255) / 256;
  if (gr > 8192) gr = 8192;
  if (gr < 1) gr = 1;
  k_gamma5<<<(unsigned)gr, 256, 0, s>>>(in, out, n);
  DD_LAUNCH_CHECK();
}

void to_half(const double2* in, __half2* out, long long n, hipStream_t s) {
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  k_to_half<<<(unsigned)g, 256, 0, s>>>(in, out, n);
  DD_LAUNCH_CHECK();
}

// one thread per site and field: largest |re|, |im| of the 12 components,
// the components divided by it rounded to FP16, and their decoded FP64 value
__global__ void k_encode_sites(const float2* __restrict__ in, __half2* __restrict__ half, float* __restrict__ scale,
                               double2* __restrict__ dec, int nblk) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15;
  if (blk >= nblk) return;
  const long long fs = (long long)nblk * 192, off = (long long)blockIdx.y * fs + (long long)blk * 192 + loc;
  float2 v[12];
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    v[c] = in[off + c * 16];
    m = fmaxf(m, fmaxf(fabsf(v[c].x), fabsf(v[c].y)));
  }
  const float inv = m > 0.f ? 1.f / m : 0.f;
  scale[(long long)blockIdx.y * nblk * 16 + (long long)blk * 16 + loc] = m;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const __half2 h = __floats2half2_rn(v[c].x * inv, v[c].y * inv);
    half[off + c * 16] = h;
    const float2 r = __half22float2(h);
    dec[off + c * 16] = make_double2((double)r.x * m, (double)r.y * m);
  }
}

void encode_sites(const FineGeom& g, const float2* in, __half2* half, float* scale, double2* dec, int nb,
                  hipStream_t s) {
  k_encode_sites<<<dim3(nblocks((size_t)g.nblk * 16, 256), nb), 256, 0, s>>>(in, half, scale, dec, g.nblk);
  DD_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_encode_h(const C<T>* __restrict__ in, __half2* __restrict__ half, float* __restrict__ scale,
                           int nblk) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15;
  if (blk >= nblk) return;
  const long long fs = (long long)nblk * 192, ss = (long long)nblk * 16, r = blockIdx.y;
  C<T> v[12];
  load_spinor<T>(in + r * fs, blk, loc, v);
  store_site<T, __half2>(half + r * fs, scale + r * ss, blk, loc, v);
}
template <typename T>
__global__ void k_decode_h(const __half2* __restrict__ half, const float* __restrict__ scale, C<T>* __restrict__ out,
                           int nblk) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15;
  if (blk >= nblk) return;
  const long long fs = (long long)nblk * 192, ss = (long long)nblk * 16, r = blockIdx.y;
  C<T> v[12];
  load_site<T, __half2>(half + r * fs, scale + r * ss, blk, loc, v);
  C<T>* o = out + r * fs + (long long)blk * 192 + loc;
#pragma unroll
  for (int c = 0; c < 12; ++c) o[c * 16] = v[c];
}
template <typename T>
void encode_h(const FineGeom& g, const C<T>* in, __half2* half, float* scale, int nb, hipStream_t s) {
  k_encode_h<T><<<dim3(nblocks((size_t)g.nblk * 16, 256), nb), 256, 0, s>>>(in, half, scale, g.nblk);
  DD_LAUNCH_CHECK();
}
template <typename T>
void decode_h(const FineGeom& g, const __half2* half, const float* scale, C<T>* out, int nb, hipStream_t s) {
  k_decode_h<T><<<dim3(nblocks((size_t)g.nblk * 16, 256), nb), 256, 0, s>>>(half, scale, out, g.nblk);
  DD_LAUNCH_CHECK();
}
template void encode_h<double>(const FineGeom&, const double2*, __half2*, float*, int, hipStream_t);
template void encode_h<float>(const FineGeom&, const float2*, __half2*, float*, int, hipStream_t);
template void decode_h<double>(const FineGeom&, const __half2*, const float*, double2*, int, hipStream_t);
template void decode_h<float>(const FineGeom&, const __half2*, const float*, float2*, int, hipStream_t);

}  // namespace ddamg
