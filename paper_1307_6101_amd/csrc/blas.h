// Vector kernels for the Krylov solvers and the MR/GMRES inner products.
// Vectors are flat arrays of n complex numbers (the layout does not matter
// for these operations).  Reductions are deterministic: per-workgroup
// partials, then one workgroup sums them in a fixed order; the result is
// always accumulated in FP64.
#pragma once

#include <complex>
#include <vector>

#include "common.h"

namespace ddamg {

constexpr int KMAX = 32;   // max vectors in one fused dot / linear combination

struct Coefs {
  double2 c[KMAX];
};

template <typename T> void vzero(C<T>* x, long long n, hipStream_t s);
template <typename TA, typename TB> void vcopy(const C<TA>* x, C<TB>* y, long long n, hipStream_t s);
// y += a x
template <typename T> void vaxpy(double2 a, const C<T>* x, C<T>* y, long long n, hipStream_t s);
// y = a y
template <typename T> void vscale(double2 a, C<T>* y, long long n, hipStream_t s);
// y = b - y
template <typename T> void vbmy(const C<T>* b, C<T>* y, long long n, hipStream_t s);
// y += sum_j c_j Z_j, Z_j = Z + j*stride (k <= KMAX)
template <typename T, typename TZ>
void vlincomb(const Coefs& c, int k, const C<TZ>* Z, long long stride, C<T>* y, long long n,
              hipStream_t s);

// y += sum_j c_j Z_j, then dst = scale * y (one pass)
template <typename T>
void vlincomb_scale(const Coefs& c, int k, const C<T>* Z, long long stride, C<T>* y, long long n,
                    double scale, C<T>* dst, hipStream_t s);

// Fused inner products <V_j, w> (j < k) and <w, w> (entry k), accumulated in
// FP64 in a fixed order; fetch() copies them to the host.
class Reducer {
 public:
  Reducer();
  ~Reducer();
  template <typename T>
  void dots(const C<T>* V, long long stride, int k, const C<T>* w, long long n, bool with_norm,
            hipStream_t s);
  // w += sum_j c_j V_j, then the inner products of the updated w (one pass)
  template <typename T>
  void update_dots(const Coefs& c, const C<T>* V, long long stride, int k, C<T>* w, long long n,
                   hipStream_t s);
  // copy the last results to the host (synchronises the stream)
  void fetch(int count, std::complex<double>* out, hipStream_t s);

 private:
  template <typename T>
  void launch(const C<T>* V, long long stride, int k, C<T>* w, long long n, bool upd, const Coefs* c,
              hipStream_t s);
  double* partial_ = nullptr;   // [GMAX][2*(KMAX+1)]
  double2* result_ = nullptr;   // [KMAX+1]
  double2* host_ = nullptr;     // pinned
};

}  // namespace ddamg
