// Shared helpers of the gfx950 DD-alpha-AMG library: complex arithmetic on
// HIP vector types, error handling, launch helpers and wavefront reductions.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <type_traits>

namespace ddamg {

// ---------------------------------------------------------------------------
// Errors.  Internal code throws ddamg::Error; the C ABI turns it into a
// status code and a thread-local message.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define DD_CHECK_HIP(call)                                                        \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::ddamg::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define DD_REQUIRE(cond, msg)                                   \
  do {                                                          \
    if (!(cond)) throw ::ddamg::Error(-1, std::string(msg));    \
  } while (0)

#define DD_LAUNCH_CHECK() DD_CHECK_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Complex numbers: double2 / float2 with (x, y) = (re, im).
// ---------------------------------------------------------------------------
template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename T> using C = typename cplx<T>::type;

template <typename T> __host__ __device__ inline C<T> mk(T re, T im) {
  C<T> c; c.x = re; c.y = im; return c;
}
template <typename T> __host__ __device__ inline C<T> czero() { return mk<T>(T(0), T(0)); }
template <typename V> __host__ __device__ inline V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }
template <typename V> __host__ __device__ inline V csub(V a, V b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename V> __host__ __device__ inline V cmul(V a, V b) {
  V c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
// conj(a) * b
template <typename V> __host__ __device__ inline V cjmul(V a, V b) {
  V c; c.x = a.x * b.x + a.y * b.y; c.y = a.x * b.y - a.y * b.x; return c;
}
template <typename V> __host__ __device__ inline V cconj(V a) { a.y = -a.y; return a; }
// fused multiply-add of one real type (host and device)
__host__ __device__ inline double rfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ inline float rfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// acc += a * b, as four fused multiply-adds into the accumulator (written
// as acc + (a.x b.x - a.y b.y) the compiler may only fuse the inner
// difference, leaving a multiply and an add besides)
template <typename V> __host__ __device__ inline void cfma(V& acc, V a, V b) {
  acc.x = rfma(a.x, b.x, acc.x);
  acc.x = rfma(-a.y, b.y, acc.x);
  acc.y = rfma(a.x, b.y, acc.y);
  acc.y = rfma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename V> __host__ __device__ inline void cjfma(V& acc, V a, V b) {
  acc.x = rfma(a.x, b.x, acc.x);
  acc.x = rfma(a.y, b.y, acc.x);
  acc.y = rfma(a.x, b.y, acc.y);
  acc.y = rfma(-a.y, b.x, acc.y);
}
template <typename V, typename S> __host__ __device__ inline V cscale(V a, S s) {
  a.x *= s; a.y *= s; return a;
}
// multiply by i
template <typename V> __host__ __device__ inline V cmuli(V a) { V c; c.x = -a.y; c.y = a.x; return c; }
template <typename V> __host__ __device__ inline V cmulmi(V a) { V c; c.x = a.y; c.y = -a.x; return c; }

// conversion between precisions
template <typename To, typename From> __host__ __device__ inline C<To> ccast(From a) {
  return mk<To>(static_cast<To>(a.x), static_cast<To>(a.y));
}

// Operator storage: the arithmetic type T reads stored complex numbers of
// type S (C<T> itself, or __half2 for FP16 storage with FP32 arithmetic).
template <typename T, typename S> struct Load;
template <> struct Load<double, double2> {
  static __device__ inline double2 f(const double2& v) { return v; }
};
template <> struct Load<float, float2> {
  static __device__ inline float2 f(const float2& v) { return v; }
};
template <> struct Load<float, __half2> {
  static __device__ inline float2 f(const __half2& v) { return __half22float2(v); }
};
template <> struct Load<double, __half2> {
  static __device__ inline double2 f(const __half2& v) {
    const float2 t = __half22float2(v);
    return make_double2(t.x, t.y);
  }
};
template <typename T, typename S> __device__ inline C<T> ldc(const S& v) { return Load<T, S>::f(v); }
// zero of a storage type (__half2's default constructor leaves it unset)
template <typename S> __device__ inline S szero();
template <> __device__ inline double2 szero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ inline float2 szero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ inline __half2 szero<__half2>() { return __float2half2_rn(0.f); }

// ---------------------------------------------------------------------------
// Wavefront-level reductions (64 lanes) within groups of `width` lanes.
// ---------------------------------------------------------------------------
template <int WIDTH, typename T> __device__ inline T group_sum(T v) {
#pragma unroll
  for (int off = WIDTH / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WIDTH);
  return v;
}

// Sum over each group of 16 lanes (a DPP row), left in every lane: swaps
// within pairs and quads, then the half-row and row mirrors, each a data
// parallel move folded into the add (no LDS round trip).
template <int CTRL> __device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ inline float row_sum16(float v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return v;
}
template <typename T> __device__ inline T sum16(T v) { return group_sum<16>(v); }
template <> __device__ inline float sum16<float>(float v) { return row_sum16(v); }

inline unsigned nblocks(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// Batches of nb right-hand sides are cut into launches that give every
// thread RB of them (4 in FP32, 2 in FP64, 1 for the rest): f(rb, first,
// nchunks) launches nchunks chunks of rb fields starting at field `first`.
template <typename T, typename F>
inline void rhs_chunks(int nb, F&& f) {
  int done = 0;
  if constexpr (sizeof(T) == 4) {
    if (nb >= 4) {
      f(std::integral_constant<int, 4>{}, 0, nb / 4);
      done = nb / 4 * 4;
    }
  }
  if (done == 0 && nb >= 2) {
    f(std::integral_constant<int, 2>{}, 0, nb / 2);
    done = nb / 2 * 2;
  }
  if (nb > done) f(std::integral_constant<int, 1>{}, done, nb - done);
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// A named range on the host timeline for tracing tools (ROCTx: rocprofv3
// --marker-trace shows each range with the kernels launched inside it);
// nearly free when no tool listens.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace ddamg
