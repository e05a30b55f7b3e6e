// Fine-lattice (level 0) data layout and launchers.
//
// Native fine layout: the lattice is cut into 2^4 blocks of 16 sites (the SAP
// blocks); inside a block, site (lx,ly,lz,lt) has local index
// lx + 2ly + 4lz + 8lt.  Blocks are numbered tile by tile: sixteen
// consecutive block numbers form a 2x2x2x2 tile of blocks (a 4^4 brick of
// sites, the aggregate shape of the first level), tiles lexicographic over
// the tile grid dims/4, blocks inside a tile in the same bit order as sites
// inside a block.  A field is stored [block][component][16 sites], so one
// 16-lane group of a wavefront reads one block, each component load is one
// contiguous segment, and a 256-thread workgroup covers one compact 4^4
// brick, whose neighbours are half as often outside it as those of a row of
// blocks.
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

// Block numbering.  The 2^4 blocks form 4^4 tiles of 2x2x2x2 blocks
// (block = 16 * tile + index in the tile); tiles are numbered in a
// Morton-like order: level by level, every direction whose remaining tile
// count is even contributes one binary digit (finest level first), and what
// is left (odd counts) is numbered lexicographically.  Consecutive tiles
// thus form compact 4-D regions in all directions, so the workgroups that
// run one after another on an XCD share their faces in its L2.
__host__ __device__ inline int tile_encode(const int nt[4], const int tc[4]) {
  int c[4] = {tc[0], tc[1], tc[2], tc[3]}, rem[4] = {nt[0], nt[1], nt[2], nt[3]};
  int idx = 0, mult = 1;
  for (;;) {
    int f[4], prod = 1;
    for (int mu = 0; mu < 4; ++mu) {
      f[mu] = (rem[mu] % 2 == 0) ? 2 : 1;
      prod *= f[mu];
    }
    if (prod == 1) break;
    const int digit = (c[0] % f[0]) + f[0] * ((c[1] % f[1]) + f[1] * ((c[2] % f[2]) + f[2] * (c[3] % f[3])));
    idx += digit * mult;
    mult *= prod;
    for (int mu = 0; mu < 4; ++mu) {
      c[mu] /= f[mu];
      rem[mu] /= f[mu];
    }
  }
  return idx + mult * (c[0] + rem[0] * (c[1] + rem[1] * (c[2] + rem[2] * c[3])));
}
__host__ __device__ inline void tile_decode(const int nt[4], int tile, int tc[4]) {
  int rem[4] = {nt[0], nt[1], nt[2], nt[3]}, scale[4] = {1, 1, 1, 1};
  for (int mu = 0; mu < 4; ++mu) tc[mu] = 0;
  for (;;) {
    int f[4], prod = 1;
    for (int mu = 0; mu < 4; ++mu) {
      f[mu] = (rem[mu] % 2 == 0) ? 2 : 1;
      prod *= f[mu];
    }
    if (prod == 1) break;
    int digit = tile % prod;
    tile /= prod;
    for (int mu = 0; mu < 4; ++mu) {
      tc[mu] += (digit % f[mu]) * scale[mu];
      digit /= f[mu];
      scale[mu] *= f[mu];
      rem[mu] /= f[mu];
    }
  }
  for (int mu = 0; mu < 4; ++mu) {
    tc[mu] += (tile % rem[mu]) * scale[mu];
    tile /= rem[mu];
  }
}
// block number of the block with coordinates b (block grid nb) and back
__host__ __device__ inline int block_encode(const int nb[4], const int b[4]) {
  const int it = (b[0] & 1) | ((b[1] & 1) << 1) | ((b[2] & 1) << 2) | ((b[3] & 1) << 3);
  const int nt[4] = {nb[0] >> 1, nb[1] >> 1, nb[2] >> 1, nb[3] >> 1};
  const int tc[4] = {b[0] >> 1, b[1] >> 1, b[2] >> 1, b[3] >> 1};
  return tile_encode(nt, tc) * 16 + it;
}
__host__ __device__ inline void block_decode(const int nb[4], int blk, int b[4]) {
  const int it = blk & 15;
  const int nt[4] = {nb[0] >> 1, nb[1] >> 1, nb[2] >> 1, nb[3] >> 1};
  int tc[4];
  tile_decode(nt, blk >> 4, tc);
  for (int mu = 0; mu < 4; ++mu) b[mu] = 2 * tc[mu] + ((it >> mu) & 1);
}
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

// out = D in in FP64 for nb fields stored in FP16 with site scales (the form
// of encode_sites): D applied to exactly the values the FP16 field stands for
void dslash_hs(const FineOpView<double>& op, const __half2* in, const float* ins, double2* out, hipStream_t s,
               int nb = 1);

// one SAP colour pass: z += MR-block-solve(b - D z) on blocks of colour c,
// for nb right-hand sides (fields as for dslash)
template <typename T, typename S>
void sap_colour(const FineOpView<T, S>& op, const int* colour_blocks, int colour, int mr_iters,
                const C<T>* b, C<T>* z, hipStream_t s, int nb = 1);

// The same pass with FP16 operator data and FP16 spinors b, z with one FP32
// scale per site (the layout of encode_sites below; bs, zs the scales); z
// is re-encoded with each updated site's new scale
void sap_colour_hs(const FineOpView<float, __half2>& op, const int* colour_blocks, int colour, int mr_iters,
                   const __half2* b, const float* bs, __half2* z, float* zs, hipStream_t s, int nb = 1);

// FP64 -> FP16 copy of n complex numbers (operator storage)
void to_half(const double2* in, __half2* out, long long n, hipStream_t s);

// FP16 fine fields with one FP32 scale per site (the largest |re|, |im| of
// the site's 12 components; entries stored divided by it), for nb fields:
// half [nb][nblk*192], scale [nb][V] (site blk*16 + loc).  encode_sites also
// writes the decoded FP64 field `dec` (the values the stored field stands
// for).
void encode_sites(const FineGeom& g, const float2* in, __half2* half, float* scale, double2* dec, int nb,
                  hipStream_t s);
// native fields at precision T <-> that FP16 form (no decoded copy)
template <typename T>
void encode_h(const FineGeom& g, const C<T>* in, __half2* half, float* scale, int nb, hipStream_t s);
template <typename T>
void decode_h(const FineGeom& g, const __half2* half, const float* scale, C<T>* out, int nb, hipStream_t s);

// out = Gamma5 in for nb native fine fields (spins 3 and 4, components
// 6..11, change sign; in == out allowed)
void gamma5(const FineGeom& g, const double2* in, double2* out, int nb, hipStream_t s);


}  // namespace ddamg
