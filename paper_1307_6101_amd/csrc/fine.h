// Fine-lattice (level 0) data layout and launchers.
//
// Native fine layout: the lattice is cut into 2^4 blocks of 16 sites (the SAP
// blocks), numbered lexicographically over the block grid dims/2; inside a
// block, site (lx,ly,lz,lt) has local index lx + 2ly + 4lz + 8lt.  A field is
// stored [block][component][16 sites], so one 16-lane group of a wavefront
// reads one block, and each component load is one contiguous segment.
//   spinor  [nblk][12][16]      component = spin*3 + colour
//   links   [nblk][4][9][16]    U_mu(x) row-major, x the site of the block
//   clover  [nblk][36][16]      per chirality 18 entries: 3 packed real
//                               diagonal pairs, 15 upper off-diagonals
// The neighbour of local site l in direction +-mu is local site l ^ (1<<mu),
// either in the same block or in the neighbouring block (table nbr_blk).
#pragma once

#include "common.h"

namespace ddamg {

struct FineGeom {
  int dims[4];
  int nb[4];        // blocks per direction (dims / 2)
  int nblk;         // number of 2^4 blocks
  long long V;      // sites
};

FineGeom make_fine_geom(const int dims[4]);
// host tables: nbr_blk[blk*8 + 2*mu + (0 fwd | 1 bwd)], colour lists
void fine_tables(const FineGeom& g, int* nbr_blk, int* colour_blocks /* [2][nblk/2] */);

template <typename T, typename S = C<T>>
struct FineOpView {
  const S* U;         // native links
  const S* A;         // native clover (mass folded in)
  const int* nbr;     // nbr_blk table
  int nblk;
};

// canonical complex128 <-> native at precision T (nrhs fields)
template <typename T>
void fine_to_native(const FineGeom& g, const double2* in, C<T>* out, int nrhs, hipStream_t s);
template <typename T>
void fine_from_native(const FineGeom& g, const C<T>* in, double2* out, int nrhs, hipStream_t s);

// links canonical complex128 -> native T
template <typename T>
void links_to_native(const FineGeom& g, const double2* links, C<T>* out, hipStream_t s);
// clover (+ (m0+4)) from canonical complex128 links, native FP64
void clover_build(const FineGeom& g, const double2* links, double m0, double csw, double2* out,
                  hipStream_t s);

// out = D in for nb native fields (field r at offset r * nblk * 192)
template <typename T, typename S>
void dslash(const FineOpView<T, S>& op, const C<T>* in, C<T>* out, hipStream_t s, int nb = 1);

// one SAP colour pass: z += MR-block-solve(b - D z) on blocks of colour c,
// for nb right-hand sides (fields as for dslash)
template <typename T, typename S>
void sap_colour(const FineOpView<T, S>& op, const int* colour_blocks, int colour, int mr_iters,
                const C<T>* b, C<T>* z, hipStream_t s, int nb = 1);

// FP64 -> FP16 copy of n complex numbers (operator storage)
void to_half(const double2* in, __half2* out, long long n, hipStream_t s);

}  // namespace ddamg
