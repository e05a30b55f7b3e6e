#include "blas.h"

namespace ddamg {

constexpr int GMAX = 512;      // max workgroups of the first reduction pass
constexpr int RED_BS = 256;

template <typename T>
__global__ void k_zero(C<T>* x, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) x[i] = czero<T>();
}
template <typename TA, typename TB>
__global__ void k_copy(const C<TA>* __restrict__ x, C<TB>* __restrict__ y, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = ccast<TB>(x[i]);
}
template <typename T>
__global__ void k_axpy(double2 a, const C<T>* __restrict__ x, C<T>* __restrict__ y, long long n) {
  const C<T> aa = ccast<T>(a);
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    C<T> v = y[i];
    cfma(v, aa, x[i]);
    y[i] = v;
  }
}
template <typename T>
__global__ void k_scale(double2 a, C<T>* __restrict__ y, long long n) {
  const C<T> aa = ccast<T>(a);
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = cmul(aa, y[i]);
}
template <typename T>
__global__ void k_bmy(const C<T>* __restrict__ b, C<T>* __restrict__ y, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = csub(b[i], y[i]);
}
template <typename T, typename TZ>
__global__ void k_lincomb(Coefs c, int k, const C<TZ>* __restrict__ Z, long long stride,
                          C<T>* __restrict__ y, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    double2 acc = ccast<double>(y[i]);
    for (int j = 0; j < k; ++j) cfma(acc, c.c[j], ccast<double>(Z[j * stride + i]));
    y[i] = ccast<T>(acc);
  }
}

static unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T> void vzero(C<T>* x, long long n, hipStream_t s) {
  k_zero<T><<<grid_for(n), 256, 0, s>>>(x, n);
  DD_LAUNCH_CHECK();
}
template <typename TA, typename TB> void vcopy(const C<TA>* x, C<TB>* y, long long n, hipStream_t s) {
  k_copy<TA, TB><<<grid_for(n), 256, 0, s>>>(x, y, n);
  DD_LAUNCH_CHECK();
}
template <typename T> void vaxpy(double2 a, const C<T>* x, C<T>* y, long long n, hipStream_t s) {
  k_axpy<T><<<grid_for(n), 256, 0, s>>>(a, x, y, n);
  DD_LAUNCH_CHECK();
}
template <typename T> void vscale(double2 a, C<T>* y, long long n, hipStream_t s) {
  k_scale<T><<<grid_for(n), 256, 0, s>>>(a, y, n);
  DD_LAUNCH_CHECK();
}
template <typename T> void vbmy(const C<T>* b, C<T>* y, long long n, hipStream_t s) {
  k_bmy<T><<<grid_for(n), 256, 0, s>>>(b, y, n);
  DD_LAUNCH_CHECK();
}
template <typename T, typename TZ>
void vlincomb(const Coefs& c, int k, const C<TZ>* Z, long long stride, C<T>* y, long long n,
              hipStream_t s) {
  if (k <= 0) return;
  DD_REQUIRE(k <= KMAX, "too many vectors in a linear combination");
  k_lincomb<T, TZ><<<grid_for(n), 256, 0, s>>>(c, k, Z, stride, y, n);
  DD_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// fused inner products
// ---------------------------------------------------------------------------
__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__global__ void __launch_bounds__(RED_BS) k_dots_pass1(const C<T>* __restrict__ V, long long stride,
                                                       int k, const C<T>* __restrict__ w, long long n,
                                                       int with_norm, double* __restrict__ partial) {
  __shared__ double lds[RED_BS / 64][2 * (KMAX + 1)];
  double acc[2 * KMAX];
  double nrm = 0;
#pragma unroll
  for (int j = 0; j < 2 * KMAX; ++j) acc[j] = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 wi = ccast<double>(w[i]);
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      if (j < k) {
        const double2 v = ccast<double>(V[j * stride + i]);
        acc[2 * j] += v.x * wi.x + v.y * wi.y;
        acc[2 * j + 1] += v.x * wi.y - v.y * wi.x;
      }
    nrm += wi.x * wi.x + wi.y * wi.y;
  }
  const int nv = 2 * (k + (with_norm ? 1 : 0));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 2 * KMAX; ++j)
    if (j < 2 * k) {
      const double s = wsum(acc[j]);
      if (lane == 0) lds[wave][j] = s;
    }
  if (with_norm) {
    const double s = wsum(nrm);
    if (lane == 0) {
      lds[wave][2 * k] = s;
      lds[wave][2 * k + 1] = 0;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    double s = 0;
    for (int q = 0; q < RED_BS / 64; ++q) s += lds[q][j];
    partial[(long long)blockIdx.x * 2 * (KMAX + 1) + j] = s;
  }
}

__global__ void k_dots_pass2(const double* __restrict__ partial, int g, int nv, double2* __restrict__ out) {
  // one thread per value, fixed summation order
  const int j = threadIdx.x;
  if (j >= nv) return;
  double s = 0;
  for (int q = 0; q < g; ++q) s += partial[(long long)q * 2 * (KMAX + 1) + j];
  reinterpret_cast<double*>(out)[j] = s;
}

Reducer::Reducer() {
  DD_CHECK_HIP(hipMalloc(&partial_, sizeof(double) * GMAX * 2 * (KMAX + 1)));
  DD_CHECK_HIP(hipMalloc(&result_, sizeof(double2) * (KMAX + 1)));
  DD_CHECK_HIP(hipHostMalloc(&host_, sizeof(double2) * (KMAX + 1), hipHostMallocDefault));
}
Reducer::~Reducer() {
  (void)hipFree(partial_);
  (void)hipFree(result_);
  (void)hipHostFree(host_);
}

template <typename T>
void Reducer::dots(const C<T>* V, long long stride, int k, const C<T>* w, long long n, bool with_norm,
                   hipStream_t s) {
  DD_REQUIRE(k <= KMAX, "too many vectors in a fused dot product");
  long long g = (n + RED_BS - 1) / RED_BS;
  if (g > GMAX) g = GMAX;
  if (g < 1) g = 1;
  k_dots_pass1<T><<<(unsigned)g, RED_BS, 0, s>>>(V, stride, k, w, n, with_norm ? 1 : 0, partial_);
  DD_LAUNCH_CHECK();
  const int nv = 2 * (k + (with_norm ? 1 : 0));
  k_dots_pass2<<<1, 128, 0, s>>>(partial_, (int)g, nv, result_);
  DD_LAUNCH_CHECK();
}

void Reducer::fetch(int count, std::complex<double>* out, hipStream_t s) {
  DD_CHECK_HIP(hipMemcpyAsync(host_, result_, sizeof(double2) * count, hipMemcpyDeviceToHost, s));
  DD_CHECK_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < count; ++j) out[j] = std::complex<double>(host_[j].x, host_[j].y);
}

#define DD_INST(T)                                                                            \
  template void vzero<T>(C<T>*, long long, hipStream_t);                                     \
  template void vaxpy<T>(double2, const C<T>*, C<T>*, long long, hipStream_t);               \
  template void vscale<T>(double2, C<T>*, long long, hipStream_t);                           \
  template void vbmy<T>(const C<T>*, C<T>*, long long, hipStream_t);                         \
  template void Reducer::dots<T>(const C<T>*, long long, int, const C<T>*, long long, bool,  \
                                 hipStream_t);
DD_INST(double)
DD_INST(float)
#undef DD_INST
template void vcopy<double, double>(const C<double>*, C<double>*, long long, hipStream_t);
template void vcopy<double, float>(const C<double>*, C<float>*, long long, hipStream_t);
template void vcopy<float, double>(const C<float>*, C<double>*, long long, hipStream_t);
template void vcopy<float, float>(const C<float>*, C<float>*, long long, hipStream_t);
template void vlincomb<double, double>(const Coefs&, int, const C<double>*, long long, C<double>*,
                                       long long, hipStream_t);
template void vlincomb<double, float>(const Coefs&, int, const C<float>*, long long, C<double>*,
                                      long long, hipStream_t);
template void vlincomb<float, float>(const Coefs&, int, const C<float>*, long long, C<float>*,
                                     long long, hipStream_t);

}  // namespace ddamg
