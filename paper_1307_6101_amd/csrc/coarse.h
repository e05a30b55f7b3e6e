// Coarse levels (l >= 1): the Galerkin operators D_{l} = P^H D_{l-1} P as
// block stencils (Sec. 1, Sec. 2), their SAP smoother, the odd-even pieces of
// the coarsest solve (Sec. 3), and the interpolation P between levels.
//
// Layout: a level-l field is [V_l][d] complex (canonical coarse site order,
// d = 2N_{l-1}, components 0..d/2-1 carry Gamma5 = +1).
// The Galerkin product produces, in FP64, the self block and the four
// forward blocks per site, [V_l][5][d][d] row-major; the backward blocks
// follow from gamma5-symmetry,
//   B_mu(x) = G5 F_mu(x - mu)^H G5,   B_mu(x)[i][j] = g_i g_j conj(F_mu(x-mu)[j][i]).
// For applying the operator each precision keeps an expanded copy with all
// nine blocks, [V_l][9][d][d], block k = self, +x,+y,+z,+t, -x,-y,-z,-t, each
// stored column-major (element (i, j) at j*d + i): one wavefront handles one
// site with lane i computing row i, so every matrix load is one contiguous
// segment across the lanes.
#pragma once

#include <vector>

#include "common.h"

namespace ddamg {

struct CoarseGeom {
  int dims[4];
  int V;
  int d;                       // complex components per site
  // host tables
  std::vector<int> nbr9;       // [V][9]: self, +x..+t, -x..-t
  // SAP blocks
  int sap[4];
  int nblk, bs;                // blocks, sites per block
  std::vector<int> blk_sites;  // [nblk][bs], blocks colour-major (colour 0 first)
  std::vector<int> site_blk;   // [V] block id
  std::vector<int> site_pos;   // [V] block id * bs + index in the block
  std::vector<unsigned> inmask;  // [nblk*bs] by block-major position: bit k, nbr9[k] lies in the site's block
  int kmax = 9;                // most set bits of any inmask (blocks one MR step reads per site)
  // parity (odd-even)
  bool bipartite;
  std::vector<int> even, odd;
};

CoarseGeom make_coarse_geom(const int dims[4], int d, const int sap[4]);


template <typename T, typename S = C<T>>
struct CoarseOpView {
  const S* K;          // [V][9][d][d], column-major blocks (stored as S)
  const int* nbr9;     // [V][9]: site itself, then +mu, then -mu neighbours
  int V, d;
};

// expand the FP64 Galerkin output [V][5][d][d] (row-major) into the
// nine-block column-major apply layout, stored as S (double2, float2, __half2)
template <typename S>
void expand_coarse(const double2* D5, const int* nbr9, int V, int d, S* K, hipStream_t s);

// out = D in for nb fields of the level (field r at offset r * V * d)
template <typename T, typename S>
void coarse_apply(const CoarseOpView<T, S>& op, const C<T>* in, C<T>* out, hipStream_t s, int nb = 1);

// Work buffers of a coarse SAP colour pass (each [nb][V][d], part
// [nb][V][4] for a batch of nb); ping-ponged by MR step.
template <typename T>
struct SapScratch {
  C<T>* rho[2] = {nullptr, nullptr};
  C<T>* q[2] = {nullptr, nullptr};
  T* part[2] = {nullptr, nullptr};
};

// device SAP tables of a level (see CoarseGeom)
struct SapTables {
  const int* blk_sites;        // [nblk][bs], blocks colour-major
  const int* site_pos;         // [V]
  const unsigned* inmask;      // [nblk*bs], by block-major position
  int nblk, bs;
  int kmax;                    // most operator blocks an MR step reads for one site
};

// one SAP colour pass z <- z + MR_blocks(b - D z) on the blocks of colour
// `colour`, for nb fields
template <typename T, typename S>
void coarse_sap_colour(const CoarseOpView<T, S>& op, const SapTables& tb, int colour, int mr_iters, const C<T>* b,
                       C<T>* z, SapScratch<T>& ws, hipStream_t s, int nb = 1);

// odd-even: out(x) = gamma in_c(x) + alpha S(x) in_s(x) + beta sum_hops(in_h)(x)
// for x in `sites` (other sites of out untouched)
template <typename T, typename S>
void coarse_site_apply(const CoarseOpView<T, S>& op, const int* sites, int nsites, T gamma,
                       const C<T>* in_c, T alpha, const C<T>* in_s, T beta, const C<T>* in_h,
                       C<T>* out, hipStream_t s, int nb = 1);
// out(x) = M(x) in(x) for x in `sites`, M = [nsites][d][d] (dense per-site
// matrices, column-major); nb fields n apart
template <typename T>
void site_matvec(const C<T>* M, const int* sites, int nsites, int d, long long n, const C<T>* in, C<T>* out,
                 hipStream_t s, int nb = 1);
// Dense Schur complement S = D_oo - D_oe D_ee^-1 D_eo (Sec. 3) of a small bipartite
// coarsest level (odd-even reduction), row-major [m][m] over the m = n_odd * d
// odd-site components; oidx[i] is the level-vector index of component i,
// eidx[i] the index of an even-site component (the two counts are equal).
// out = S in on the odd components and 0 on the even ones; nb fields n apart
template <typename T>
void dense_schur_apply(const C<T>* S, int m, const int* oidx, const int* eidx, long long n, const C<T>* in,
                       C<T>* out, hipStream_t s, int nb = 1);
// nbc level vectors n apart, vector r the unit vector of odd component j0 + r
void schur_unit_cols(double2* e, long long n, int nbc, const int* oidx, int j0, hipStream_t s);
// columns j0 .. j0 + nbc - 1 of S from the odd components of nbc level vectors
void schur_gather_cols(const double2* cols, long long n, int nbc, const int* oidx, int m, int j0, double2* S,
                       hipStream_t s);
// inverses of the self blocks (taken from the FP64 [V][5][d][d] Galerkin
// output) of `sites`, FP64 Gauss-Jordan with partial pivoting; written
// column-major, [nsites][d][d]
// *flag (device) is set to 1 when a pivot is zero or not finite
void self_block_inverse(const double2* D, const int* sites, int nsites, int d, double2* inv, int* flag,
                        hipStream_t s);

// canonical copy [V][9][d][d] row-major (self, +x..+t, -x..-t) of the FP64
// nine-block operator
void export_coarse(const CoarseOpView<double>& op, double2* out, hipStream_t s);

}  // namespace ddamg
