// Coarse levels (l >= 1): the Galerkin operators D_{l} = P^H D_{l-1} P as
// block stencils (Sec. 1, Sec. 2), their SAP smoother, the odd-even pieces of
// the coarsest solve (Sec. 3), and the interpolation P between levels.
//
// Layout: a level-l field is [V_l][d] complex (canonical coarse site order,
// d = 2N_{l-1}, components 0..d/2-1 carry Gamma5 = +1).  The operator stores
// per site the self block and the four forward blocks, [V_l][5][d][d]
// row-major; the backward block follows from gamma5-symmetry,
//   B_mu(x) = G5 F_mu(x - mu)^H G5,   B_mu(x)[i][j] = g_i g_j conj(F_mu(x-mu)[j][i]),
// so 5 of the 9 blocks are read per site.
#pragma once

#include <vector>

#include "common.h"

namespace ddamg {

struct CoarseGeom {
  int dims[4];
  int V;
  int d;                       // complex components per site
  // host tables
  std::vector<int> nbr;        // [V][8]: 2*mu + (0 fwd | 1 bwd)
  // SAP blocks
  int sap[4];
  int nblk, bs;                // blocks, sites per block
  std::vector<int> blk_sites;  // [nblk][bs], blocks colour-major (colour 0 first)
  std::vector<int> site_blk;   // [V] block id
  std::vector<int> site_loc;   // [V] position inside its block
  // parity (odd-even)
  bool bipartite;
  std::vector<int> even, odd;
};

CoarseGeom make_coarse_geom(const int dims[4], int d, const int sap[4]);

struct CoarseDev {             // device copies of the tables
  int* nbr = nullptr;
  int* blk_sites = nullptr;
  int* site_blk = nullptr;
  int* site_loc = nullptr;
  int* even = nullptr;
  int* odd = nullptr;
};

template <typename T>
struct CoarseOpView {
  const C<T>* D;       // [V][5][d][d]
  const int* nbr;
  int V, d;
};

template <typename T>
void coarse_apply(const CoarseOpView<T>& op, const C<T>* in, C<T>* out, hipStream_t s);

// one SAP colour pass on a coarse level
template <typename T>
void coarse_sap_colour(const CoarseOpView<T>& op, const int* blk_sites, const int* site_blk,
                       const int* site_loc, int nblk, int bs, int colour, int mr_iters,
                       const C<T>* b, C<T>* z, hipStream_t s);

// odd-even: out(x) = gamma in_c(x) + alpha S(x) in_s(x) + beta sum_hops(in_h)(x)
// for x in `sites` (other sites of out untouched)
template <typename T>
void coarse_site_apply(const CoarseOpView<T>& op, const int* sites, int nsites, T gamma,
                       const C<T>* in_c, T alpha, const C<T>* in_s, T beta, const C<T>* in_h,
                       C<T>* out, hipStream_t s);
// out(x) = M(x) in(x) for x in `sites`, M = [nsites][d][d] (dense per-site matrices)
template <typename T>
void site_matvec(const C<T>* M, const int* sites, int nsites, int d, const C<T>* in, C<T>* out,
                 hipStream_t s);
// inverses of the self blocks of `sites` (FP64, Gauss-Jordan with partial pivoting)
void self_block_inverse(const double2* D, const int* sites, int nsites, int d, double2* inv,
                        hipStream_t s);

// canonical copy [V][9][d][d] (self, +x..+t, -x..-t) of an FP64 coarse operator
void export_coarse(const CoarseOpView<double>& op, double2* out, hipStream_t s);

}  // namespace ddamg
