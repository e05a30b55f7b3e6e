#include "blas.h"
#include "fine_dev.h"

namespace ddamg {

// max workgroups of the first reduction pass: eight per compute unit, so
// that enough wavefronts stream the vectors to keep HBM busy
constexpr int GMAX = 2048;
constexpr int RED_BS = 256;
constexpr int RED_BS_ONE = 512;               // single-workgroup reduction
constexpr long long RED_ONE_MAX = 32768;      // longest vector reduced by one workgroup

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
__global__ void k_bmy(const C<T>* __restrict__ b, C<T>* __restrict__ y, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = csub(b[i], y[i]);
}
template <typename T>
__global__ void k_add(const C<T>* __restrict__ x, C<T>* __restrict__ y, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = cadd(y[i], x[i]);
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
template <typename T> void vbmy(const C<T>* b, C<T>* y, long long n, hipStream_t s) {
  k_bmy<T><<<grid_for(n), 256, 0, s>>>(b, y, n);
  DD_LAUNCH_CHECK();
}
template <typename T> void vadd(const C<T>* x, C<T>* y, long long n, hipStream_t s) {
  k_add<T><<<grid_for(n), 256, 0, s>>>(x, y, n);
  DD_LAUNCH_CHECK();
}
// ---------------------------------------------------------------------------
// fused inner products: <V_j, w> for j < k and optionally <w, w>, FP64
// accumulation.  With `upd`, the kernel first updates w += sum_j c_j V_j
// element by element and takes the inner products of the updated w (the
// second pass of classical Gram-Schmidt with re-orthogonalisation).
// A per-workgroup first pass (skipped second pass when one workgroup covers
// the vector) and a parallel second pass.
// ---------------------------------------------------------------------------
__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int BS, int KK>
__device__ inline void dots_body(const C<T>* __restrict__ V, long long stride, C<T>* __restrict__ w,
                                 long long n, bool upd, bool store, const Coefs& c, double* __restrict__ dst) {
  constexpr int k = KK;
  __shared__ double lds[BS / 64][2 * (KMAX + 1)];
  double acc[2 * KK + 1];
  double nrm = 0;
#pragma unroll
  for (int j = 0; j < 2 * KK + 1; ++j) acc[j] = 0;
  const long long S = (long long)gridDim.x * blockDim.x;
  long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if constexpr (KK <= 12) {
    // two elements per trip, all their loads issued before the arithmetic
    // (more memory requests in flight per wavefront)
    for (; i0 + S < n; i0 += 2 * S) {
      const long long i1 = i0 + S;
      double2 w0 = ccast<double>(w[i0]), w1 = ccast<double>(w[i1]);
      double2 v0[KK > 0 ? KK : 1], v1[KK > 0 ? KK : 1];
#pragma unroll
      for (int j = 0; j < KK; ++j) {
        v0[j] = ccast<double>(V[j * stride + i0]);
        v1[j] = ccast<double>(V[j * stride + i1]);
      }
      if (upd) {
#pragma unroll
        for (int j = 0; j < KK; ++j) {
          cfma(w0, c.c[j], v0[j]);
          cfma(w1, c.c[j], v1[j]);
        }
        const C<T> t0 = ccast<T>(w0), t1 = ccast<T>(w1);
        if (store) {
          w[i0] = t0;
          w[i1] = t1;
        }
        w0 = ccast<double>(t0);
        w1 = ccast<double>(t1);
      }
#pragma unroll
      for (int j = 0; j < KK; ++j) {
        acc[2 * j] += v0[j].x * w0.x + v0[j].y * w0.y + v1[j].x * w1.x + v1[j].y * w1.y;
        acc[2 * j + 1] += v0[j].x * w0.y - v0[j].y * w0.x + v1[j].x * w1.y - v1[j].y * w1.x;
      }
      nrm += w0.x * w0.x + w0.y * w0.y + w1.x * w1.x + w1.y * w1.y;
    }
  }
  for (long long i = i0; i < n; i += S) {
    double2 wi = ccast<double>(w[i]);
    if (upd) {
#pragma unroll
      for (int j = 0; j < KK; ++j) cfma(wi, c.c[j], ccast<double>(V[j * stride + i]));
      const C<T> wt = ccast<T>(wi);
      if (store) w[i] = wt;
      wi = ccast<double>(wt);
    }
#pragma unroll
    for (int j = 0; j < KK; ++j) {
      const double2 v = ccast<double>(V[j * stride + i]);
      acc[2 * j] += v.x * wi.x + v.y * wi.y;
      acc[2 * j + 1] += v.x * wi.y - v.y * wi.x;
    }
    nrm += wi.x * wi.x + wi.y * wi.y;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 2 * KK; ++j) {
    const double sj = wsum(acc[j]);
    if (lane == 0) lds[wave][j] = sj;
  }
  {
    const double sn = wsum(nrm);
    if (lane == 0) {
      lds[wave][2 * k] = sn;
      lds[wave][2 * k + 1] = 0;
    }
  }
  __syncthreads();
  const int nv = 2 * (k + 1);
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    double sj = 0;
    for (int q = 0; q < BS / 64; ++q) sj += lds[q][j];
    dst[j] = sj;
  }
}

// ---------------------------------------------------------------------------
// batched kernels (blockIdx.y = system of the batch)
// ---------------------------------------------------------------------------
template <typename T, typename TZ>
__global__ void k_blincomb(const BArg a, int k, const C<TZ>* __restrict__ Z, long long zstride,
                           C<T>* __restrict__ y, long long n, C<T>* __restrict__ dst) {
  const int r = blockIdx.y;
  Z += (long long)r * n;
  y += (long long)r * n;
  const double sc = dst ? a.scale(r) : 0.0;
  if (dst) dst += (long long)r * n;
  const long long S = (long long)gridDim.x * blockDim.x;
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  // two elements per trip (two independent load streams per vector)
  for (; i + S < n; i += 2 * S) {
    double2 acc0 = ccast<double>(y[i]), acc1 = ccast<double>(y[i + S]);
    for (int j = 0; j < k; ++j) {
      const double2 cj = a.coef(r, j);
      cfma(acc0, cj, ccast<double>(Z[j * zstride + i]));
      cfma(acc1, cj, ccast<double>(Z[j * zstride + i + S]));
    }
    const C<T> v0 = ccast<T>(acc0), v1 = ccast<T>(acc1);
    if (dst) {
      dst[i] = sc == 0.0 ? czero<T>() : ccast<T>(cscale(ccast<double>(v0), sc));
      dst[i + S] = sc == 0.0 ? czero<T>() : ccast<T>(cscale(ccast<double>(v1), sc));
    } else {
      y[i] = v0;
      y[i + S] = v1;
    }
  }
  for (; i < n; i += S) {
    double2 acc = ccast<double>(y[i]);
    for (int j = 0; j < k; ++j) cfma(acc, a.coef(r, j), ccast<double>(Z[j * zstride + i]));
    const C<T> v = ccast<T>(acc);
    // with dst the updated y is only an intermediate: not written back
    if (dst) dst[i] = sc == 0.0 ? czero<T>() : ccast<T>(cscale(ccast<double>(v), sc));
    else y[i] = v;
  }
}

template <typename T, typename TZ>
void blincomb(const BArg& a, int k, const C<TZ>* Z, long long zstride, C<T>* y, long long n, int nb, C<T>* dst,
              hipStream_t s) {
  DD_REQUIRE(k >= 0 && k <= KMAX && nb >= 1 && nb <= NBMAX, "bad batched linear combination");
  long long g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  k_blincomb<T, TZ><<<dim3((unsigned)g, nb), 256, 0, s>>>(a, k, Z, zstride, y, n, dst);
  DD_LAUNCH_CHECK();
}

__global__ void k_blincomb_sites(const BArg a, int k, const __half2* __restrict__ Z, const float* __restrict__ scale,
                                 double2* __restrict__ y, int nblk, int nb) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15, r = blockIdx.y;
  if (blk >= nblk) return;
  const long long fs = (long long)nblk * 192, ss = (long long)nblk * 16;
  const long long off = (long long)r * fs + (long long)blk * 192 + loc;
  double2 acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = y[off + c * 16];
  for (int j = 0; j < k; ++j) {
    const double2 cj = a.coef(r, j);
    const double m = scale[((long long)j * nb + r) * ss + (long long)blk * 16 + loc];
    const __half2* zp = Z + (long long)j * nb * fs + off;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float2 h = __half22float2(zp[c * 16]);
      cfma(acc[c], cj, make_double2((double)h.x * m, (double)h.y * m));
    }
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) y[off + c * 16] = acc[c];
}

void blincomb_sites(const BArg& a, int k, const __half2* Z, const float* scale, double2* y, int nblk, int nb,
                    hipStream_t s) {
  DD_REQUIRE(k >= 0 && k <= KMAX && nb >= 1 && nb <= NBMAX, "bad batched linear combination");
  k_blincomb_sites<<<dim3(nblocks((size_t)nblk * 16, 256), nb), 256, 0, s>>>(a, k, Z, scale, y, nblk, nb);
  DD_LAUNCH_CHECK();
}

// The next basis vector of the outer FGMRES and its FP16 form in one pass:
// per site, dst = sc (y + sum_j c_j Z_j) as k_blincomb forms it, written in
// FP64 and encoded with the site's scale as encode_h would from dst
__global__ void k_blincomb_encode(const BArg a, int k, const double2* __restrict__ Z, long long zstride,
                                  const double2* __restrict__ y, double2* __restrict__ dst, __half2* __restrict__ half,
                                  float* __restrict__ hscale, int nblk) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = tid >> 4, loc = tid & 15, r = blockIdx.y;
  if (blk >= nblk) return;
  const long long fs = (long long)nblk * 192, ss = (long long)nblk * 16;
  const long long off = (long long)r * fs + (long long)blk * 192 + loc;
  double2 acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = y[off + c * 16];
  for (int j = 0; j < k; ++j) {
    const double2 cj = a.coef(r, j);
#pragma unroll
    for (int c = 0; c < 12; ++c) cfma(acc[c], cj, Z[j * zstride + off + c * 16]);
  }
  const double sc = a.scale(r);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    acc[c] = sc == 0.0 ? czero<double>() : cscale(acc[c], sc);
    dst[off + c * 16] = acc[c];
  }
  store_site<double, __half2>(half + (long long)r * fs, hscale + (long long)r * ss, blk, loc, acc);
}

void blincomb_encode(const BArg& a, int k, const double2* Z, long long zstride, const double2* y, double2* dst,
                     __half2* half, float* hscale, int nblk, int nb, hipStream_t s) {
  DD_REQUIRE(k >= 0 && k <= KMAX && nb >= 1 && nb <= NBMAX, "bad batched linear combination");
  k_blincomb_encode<<<dim3(nblocks((size_t)nblk * 16, 256), nb), 256, 0, s>>>(a, k, Z, zstride, y, dst, half,
                                                                             hscale, nblk);
  DD_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_bscale(const BArg a, const C<T>* __restrict__ src, C<T>* __restrict__ dst, long long n) {
  const int r = blockIdx.y;
  const double sc = a.scale(r);
  src += (long long)r * n;
  dst += (long long)r * n;
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = sc == 0.0 ? czero<T>() : ccast<T>(cscale(ccast<double>(src[i]), sc));
}

template <typename T>
void bscale(const BArg& a, const C<T>* src, C<T>* dst, long long n, int nb, hipStream_t s) {
  DD_REQUIRE(nb >= 1 && nb <= NBMAX, "batch too large");
  long long g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  k_bscale<T><<<dim3((unsigned)g, nb), 256, 0, s>>>(a, src, dst, n);
  DD_LAUNCH_CHECK();
}

template <typename T, int KK, int BS>
__global__ void __launch_bounds__(BS) k_bdots_pass1(const BArg a, int upd, const C<T>* __restrict__ V,
                                                    long long vstride, C<T>* __restrict__ w, long long n,
                                                    double* __restrict__ partial, int g) {
  const int r = blockIdx.y;
  Coefs cc;
  if (upd) {
#pragma unroll
    for (int j = 0; j < KK; ++j) cc.c[j] = a.coef(r, j);
  }
  dots_body<T, BS, KK>(V + (long long)r * n, vstride, w + (long long)r * n, n, upd != 0, upd == 1, cc,
                       partial + ((long long)r * g + blockIdx.x) * 2 * (KMAX + 1));
}

template <typename T, int KK>
struct BDotsLaunch {
  static void go(int k, unsigned g, int bs, int nb, hipStream_t s, const BArg& a, int upd, const C<T>* V,
                 long long vstride, C<T>* w, long long n, double* out) {
    if (k == KK) {
      if (bs == RED_BS_ONE)
        k_bdots_pass1<T, KK, RED_BS_ONE><<<dim3(g, nb), RED_BS_ONE, 0, s>>>(a, upd, V, vstride, w, n, out, (int)g);
      else
        k_bdots_pass1<T, KK, RED_BS><<<dim3(g, nb), RED_BS, 0, s>>>(a, upd, V, vstride, w, n, out, (int)g);
      return;
    }
    BDotsLaunch<T, KK + 1>::go(k, g, bs, nb, s, a, upd, V, vstride, w, n, out);
  }
};
template <typename T>
struct BDotsLaunch<T, KMAX + 1> {
  static void go(int, unsigned, int, int, hipStream_t, const BArg&, int, const C<T>*, long long, C<T>*, long long,
                 double*) {}
};

// second pass per system: block r reduces the g partial rows of system r
__global__ void __launch_bounds__(256) k_bdots_pass2(const double* __restrict__ partial, int g, int nv,
                                                     double* __restrict__ out) {
  __shared__ double lds[4][2 * (KMAX + 1)];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, r = blockIdx.x;
  const double* pr = partial + (long long)r * g * 2 * (KMAX + 1);
  for (int j = 0; j < nv; ++j) {
    double v = 0.0;
    for (int q = t; q < g; q += 256) v += pr[(long long)q * 2 * (KMAX + 1) + j];
    const double sv = wsum(v);
    if (lane == 0) lds[wave][j] = sv;
  }
  __syncthreads();
  if (t < nv) out[(long long)r * 2 * (KMAX + 1) + t] = lds[0][t] + lds[1][t] + lds[2][t] + lds[3][t];
}

template <typename T>
void Reducer::bdots(const BArg* a, const C<T>* V, long long vstride, int k, C<T>* w, long long n, int nb,
                    hipStream_t s, double2* dev_out, bool store_w) {
  DD_REQUIRE(k >= 0 && k <= KMAX && nb >= 1 && nb <= NBMAX, "bad batched inner products");
  // short vectors (the coarse levels): one workgroup of RED_BS_ONE threads
  // per system writes the result directly, no second pass
  const bool one = n <= RED_ONE_MAX;
  long long g = one ? 1 : (n + RED_BS * 4 - 1) / (RED_BS * 4);
  if (g > GMAX) g = GMAX;
  if (g < 1) g = 1;
  double* out = reinterpret_cast<double*>(dev_out ? dev_out : result_);
  static const BArg none{};
  BDotsLaunch<T, 0>::go(k, (unsigned)g, one ? RED_BS_ONE : RED_BS, nb, s, a ? *a : none, a ? (store_w ? 1 : 2) : 0,
                        V, vstride,
                        w, n, g == 1 ? out : partial_.p);
  DD_LAUNCH_CHECK();
  if (g > 1) {
    k_bdots_pass2<<<nb, 256, 0, s>>>(partial_.p, (int)g, 2 * (k + 1), out);
    DD_LAUNCH_CHECK();
  }
}

void Reducer::bfetch(int k1, int nb, std::complex<double>* out, hipStream_t s) {
  DD_CHECK_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < nb; ++r)
    for (int j = 0; j < k1; ++j)
      out[r * k1 + j] = std::complex<double>(host_[r * (KMAX + 1) + j].x, host_[r * (KMAX + 1) + j].y);
}

BArg Reducer::upload(const std::vector<std::complex<double>>& c, const std::vector<double>& scale, int nb,
                     hipStream_t s) {
  DD_REQUIRE(nb >= 1 && nb <= NBMAX, "batch too large");
  BArg a;
  auto cval = [&](int r, int j) {
    const size_t e = (size_t)r * KMAX + j;
    return e < c.size() ? make_double2(c[e].real(), c[e].imag()) : make_double2(0, 0);
  };
  auto sval = [&](int r) { return (size_t)r < scale.size() ? scale[r] : 0.0; };
  if (nb <= NBINL) {
    a.inl = 1;
    for (int r = 0; r < NBINL; ++r) {
      for (int j = 0; j < KMAX; ++j) a.ic[r * KMAX + j] = r < nb ? cval(r, j) : make_double2(0, 0);
      a.isc[r] = r < nb ? sval(r) : 0.0;
    }
    return a;
  }
  // slot layout: scales [NBMAX] then coefficients [nb][KMAX]; only the used
  // part is copied
  const size_t sbytes = sizeof(double) * NBMAX, slot = sbytes + sizeof(double2) * KMAX * NBMAX;
  const int k = cslot_;
  cslot_ = (cslot_ + 1) % NSLOT;
  // the staging slot is free once the copy that last used it has run
  if (cev_used_[k]) DD_CHECK_HIP(hipEventSynchronize(cev_[k]));
  unsigned char* hst = cstage_ + (size_t)k * slot;
  unsigned char* dvc = cdev_.p + (size_t)k * slot;
  double* hs = reinterpret_cast<double*>(hst);
  double2* hc = reinterpret_cast<double2*>(hst + sbytes);
  for (int r = 0; r < nb; ++r) {
    hs[r] = sval(r);
    for (int j = 0; j < KMAX; ++j) hc[(size_t)r * KMAX + j] = cval(r, j);
  }
  DD_CHECK_HIP(hipMemcpyAsync(dvc, hst, sbytes + sizeof(double2) * KMAX * nb, hipMemcpyHostToDevice, s));
  DD_CHECK_HIP(hipEventRecord(cev_[k], s));
  cev_used_[k] = true;
  a.sc = reinterpret_cast<const double*>(dvc);
  a.c = reinterpret_cast<const double2*>(dvc + sbytes);
  return a;
}

Reducer::Reducer() {
  partial_.alloc((size_t)NBMAX * GMAX * 2 * (KMAX + 1));
  const size_t slot = sizeof(double2) * KMAX * NBMAX + sizeof(double) * NBMAX;
  cdev_.alloc(slot * NSLOT);
  // sizing a workspace: the device arrays above are all that is counted
  if (counting_only()) return;
  // the final sums are written by the kernels straight into coherent pinned
  // host memory: after the stream synchronisation the host reads them with
  // no copy in between
  DD_CHECK_HIP(hipHostMalloc(&host_, sizeof(double2) * NBMAX * (KMAX + 1), hipHostMallocCoherent));
  DD_CHECK_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&result_), host_, 0));
  DD_CHECK_HIP(hipHostMalloc(&cstage_, slot * NSLOT, hipHostMallocDefault));
  for (int k = 0; k < NSLOT; ++k) DD_CHECK_HIP(hipEventCreateWithFlags(&cev_[k], hipEventDisableTiming));
}
Reducer::~Reducer() {
  for (int k = 0; k < NSLOT; ++k)
    if (cev_[k]) (void)hipEventDestroy(cev_[k]);
  if (host_) (void)hipHostFree(host_);
  if (cstage_) (void)hipHostFree(cstage_);
}

#define DD_INST(T)                                                                            \
  template void vzero<T>(C<T>*, long long, hipStream_t);                                     \
  template void vbmy<T>(const C<T>*, C<T>*, long long, hipStream_t);                         \
  template void vadd<T>(const C<T>*, C<T>*, long long, hipStream_t);                         \
  template void Reducer::bdots<T>(const BArg*, const C<T>*, long long, int, C<T>*, long long, int, \
                                  hipStream_t, double2*, bool);                                \
  template void blincomb<T, T>(const BArg&, int, const C<T>*, long long, C<T>*, long long, int, C<T>*, \
                               hipStream_t);                                               \
  template void bscale<T>(const BArg&, const C<T>*, C<T>*, long long, int, hipStream_t);
DD_INST(double)
DD_INST(float)
#undef DD_INST
template void vcopy<double, double>(const C<double>*, C<double>*, long long, hipStream_t);
template void vcopy<double, float>(const C<double>*, C<float>*, long long, hipStream_t);
template void vcopy<float, double>(const C<float>*, C<double>*, long long, hipStream_t);
template void vcopy<float, float>(const C<float>*, C<float>*, long long, hipStream_t);
template void blincomb<double, float>(const BArg&, int, const C<float>*, long long, C<double>*, long long, int,
                                      C<double>*, hipStream_t);

}  // namespace ddamg
