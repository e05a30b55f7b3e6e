// Aggregation-based interpolation P_l: level l -> level l+1 (Sec. 1: P groups
// spins 1,2 and spins 3,4 separately, R = P^H; Sec. 2.2 / Alg. 3, Alg. 4:
// P_l built from the test vectors; Tab. 1: aggregates of 4^4 on the fine
// level and 2^4 below).
//
// P_l is stored as N fields in the layout of level l: column k of every
// (aggregate, chirality) block V_{A,sigma} sits in field k on the sites of A
// and the components of sigma.  A coarse site is an aggregate (canonical
// order of the coarse lattice); coarse component sigma*N + k.
#pragma once

#include <vector>

#include "coarse.h"
#include "fine.h"

namespace ddamg {

struct AggTables {
  int agg[4];
  int nagg;          // aggregates = coarse sites
  int asz;           // sites per aggregate
  // fine level: members are 2^4 blocks (asz/16 per aggregate); coarse: sites
  std::vector<int> members;    // [nagg][asz/16 or asz]
  std::vector<int> member_agg; // [nblk or V] aggregate of each member
  int cdims[4];
};

AggTables make_fine_agg(const FineGeom& g, const int agg[4]);
AggTables make_coarse_agg(const CoarseGeom& g, const int agg[4]);

struct AggDev {
  int* members = nullptr;
  int* member_agg = nullptr;
};

// restriction out = P^H in and prolongation out += P in for nb right-hand
// sides (fields of the batch contiguous, each of the length of its level)
// (P stored as S: C<T>, or __half2 with T = float)
template <typename T, typename S>
void restrict_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const S* P,
                   const C<T>* in, C<T>* out, hipStream_t s, int nb = 1);
template <typename T, typename S>
void prolong_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const S* P,
                  const C<T>* in, C<T>* out, hipStream_t s, int nb = 1);
// the same with FP16 fine spinors with one FP32 scale per site (the form of
// encode_sites) and FP16 interpolation: restriction reads them, prolongation
// writes out = P in (it does not add) with new site scales
void restrict_fine_hs(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const __half2* P,
                      const __half2* in, const float* ins, float2* out, hipStream_t s, int nb);
void prolong_fine_hs(const FineGeom& g, const AggTables& a, const AggDev& ad, int N, const __half2* P,
                     const float2* in, __half2* out, float* outs, hipStream_t s, int nb);
template <typename T, typename S>
void restrict_coarse(const AggTables& a, const AggDev& ad, int d, int N, long long V,
                     const S* P, const C<T>* in, C<T>* out, hipStream_t s, int nb = 1);
template <typename T, typename S>
void prolong_coarse(const AggTables& a, const AggDev& ad, int d, int N, long long V, const S* P,
                    const C<T>* in, C<T>* out, hipStream_t s, int nb = 1);

// orthonormalise the N test-vector fields tv (FP64, layout of level l) per
// (aggregate, chirality) in index order (Gram-Schmidt with one
// re-orthogonalisation pass); result written to P.  *flag (device) is set
// to 1 where a vector is dependent on the earlier ones of its aggregate to
// within the rounding level of the Gram matrix.
void orthonormalise_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N,
                         const double2* tv, double2* P, int* flag, hipStream_t s);
void orthonormalise_coarse(const AggTables& a, const AggDev& ad, int d, int N, long long V,
                           const double2* tv, double2* P, int* flag, hipStream_t s);

// Galerkin D_{l+1} = P^H D_l P in FP64: self and forward blocks, [nagg][5][2N][2N]
void galerkin_fine(const FineGeom& g, const AggTables& a, const AggDev& ad, int N,
                   const FineOpView<double>& op, const double2* P, double2* Dc, hipStream_t s);
// cols: operator entries applied to 1 or 4 columns per workgroup (0: four
// where the level has aggregates enough to fill the device with a quarter
// of the workgroups, else one)
void galerkin_coarse(const CoarseGeom& cg, const AggTables& a, const AggDev& ad, int N,
                     const CoarseOpView<double>& op, const double2* P, double2* Dc, hipStream_t s,
                     int cols = 0);

}  // namespace ddamg
