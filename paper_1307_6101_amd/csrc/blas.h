// Vector kernels for the Krylov solvers and the MR/GMRES inner products.
// Vectors are flat arrays of n complex numbers (the layout does not matter
// for these operations).  Reductions are deterministic: per-workgroup
// partials, then one workgroup sums them in a fixed order; the result is
// always accumulated in FP64.
#pragma once

#include <complex>
#include <vector>

#include "common.h"
#include "memory.h"

namespace ddamg {

constexpr int KMAX = 32;   // max vectors in one fused dot / linear combination

struct Coefs {
  double2 c[KMAX];
};

template <typename T> void vzero(C<T>* x, long long n, hipStream_t s);
template <typename TA, typename TB> void vcopy(const C<TA>* x, C<TB>* y, long long n, hipStream_t s);
// y = b - y
template <typename T> void vbmy(const C<T>* b, C<T>* y, long long n, hipStream_t s);
// y += x
template <typename T> void vadd(const C<T>* x, C<T>* y, long long n, hipStream_t s);

// Batches: nb systems advance together; field r of a batched vector w sits
// at w + r*n, basis vector j of system r at V + j*vstride + r*n.
constexpr int NBMAX = 32;  // largest batch of the batched vector kernels
constexpr int NBINL = 4;   // batches up to this size pass their coefficients by value

// Per-system coefficients c[r][j] (r < nb, j < KMAX) and scales sc[r] of a
// batched call: in the kernel arguments for small batches, else in a
// device slot filled by Reducer::upload.
struct BArg {
  const double2* c = nullptr;
  const double* sc = nullptr;
  int inl = 0;
  double2 ic[NBINL * KMAX];
  double isc[NBINL];
  __device__ double2 coef(int r, int j) const { return inl ? ic[r * KMAX + j] : c[(size_t)r * KMAX + j]; }
  __device__ double scale(int r) const { return inl ? isc[r] : sc[r]; }
};

// y_r += sum_j c[r][j] Z_{j,r} (j < k); with dst != nullptr instead
// dst_r = sc[r] * (y_r + sum_j c[r][j] Z_{j,r}) (0 where sc[r] == 0) and y
// is left as it was (the Gram-Schmidt update of the next basis vector, whose
// intermediate is not needed)
template <typename T, typename TZ>
void blincomb(const BArg& a, int k, const C<TZ>* Z, long long zstride, C<T>* y, long long n, int nb, C<T>* dst,
              hipStream_t s);

// dst_r = sc[r] * (y_r + sum_j c[r][j] Z_{j,r}) for native fine fields
// (systems nblk*192 apart) and, in the same pass, its FP16 form with one FP32
// scale per site (half [nb][nblk*192], hscale [nb][nblk*16]), as encode_h
// would make it from dst
void blincomb_encode(const BArg& a, int k, const double2* Z, long long zstride, const double2* y, double2* dst,
                     __half2* half, float* hscale, int nblk, int nb, hipStream_t s);

// y_r += sum_j c[r][j] Z_{j,r} for fine fields stored in FP16 with one FP32
// scale per site (half [k][nb][nblk*192], scale [k][nb][nblk*16])
void blincomb_sites(const BArg& a, int k, const __half2* Z, const float* scale, double2* y, int nblk, int nb,
                    hipStream_t s);

// dst_r = sc[r] * src_r (zero where sc[r] == 0); src may equal dst
template <typename T>
void bscale(const BArg& a, const C<T>* src, C<T>* dst, long long n, int nb, hipStream_t s);

// Fused inner products <V_j, w> (j < k) and <w, w> (entry k), accumulated in
// FP64 in a fixed order, for every system r of a batch (results [nb][k+1]).
class Reducer {
 public:
  Reducer();
  ~Reducer();
  // batched: a == nullptr for plain inner products, else the update
  // w_r += sum_j c[r][j] V_{j,r} first, written back to w unless store_w is
  // false (then the products are those of the updated w, which stays as it was)
  // (results to `out` in device memory, same layout, when it is given;
  // no host access then, so the call can be captured into a graph)
  template <typename T>
  void bdots(const BArg* a, const C<T>* V, long long vstride, int k, C<T>* w, long long n, int nb,
             hipStream_t s, double2* out = nullptr, bool store_w = true);
  // results of the last batched call, out[r * (k+1) + j] (synchronises)
  void bfetch(int k1, int nb, std::complex<double>* out, hipStream_t s);
  // the coefficients (row r: system r, KMAX per row; missing entries 0) and
  // scales of a batched call; device slots stay valid for the next 63 calls
  BArg upload(const std::vector<std::complex<double>>& c, const std::vector<double>& scale, int nb,
              hipStream_t s);
 private:
  DevArray<double> partial_;    // [NBMAX][GMAX][2*(KMAX+1)]
  double2* result_ = nullptr;   // [NBMAX][KMAX+1], device alias of host_
  double2* host_ = nullptr;     // coherent pinned host memory
  // coefficient ring: pinned staging and device slots, an event per slot
  static constexpr int NSLOT = 64;
  unsigned char* cstage_ = nullptr;
  DevArray<unsigned char> cdev_;
  hipEvent_t cev_[NSLOT] = {};
  bool cev_used_[NSLOT] = {};
  int cslot_ = 0;
};

}  // namespace ddamg
